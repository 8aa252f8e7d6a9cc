// lm_kernels.hip -- gfx950 kernels of the N-particle Euler-Poincare landmark shooter.
//
// The hot path is the pair sum of the N-particle system (equation "N-particle"):
//     v_i = sum_j G(|q_i - q_j|) p_j                       (velocity, j = i included)
//     f_i = sum_{j != i} (p_i . p_j) w(|q_i - q_j|) (q_i - q_j),  w = -G'(r)/r  (force)
// evaluated once per Runge-Kutta stage.  It is bound by vector ALU issue (a pair costs
// about 45 VALU instructions in double precision and touches no memory), not by HBM, and
// it is not a dense contraction, so it runs on the vector units rather than on MFMA.
// This file holds the one-sided kernel (each target sums over all sources), used in single
// precision, with targets other than the sources, and for double-precision sets below the
// symmetric kernel's size rule (lm_sym.hip evaluates each unordered pair once); the finish
// kernel that adds either kernel's partial sums; the batched kernels; reductions and sorts.
//
// Work decomposition.  A workgroup owns a tile of 64 targets i, one per lane, and
// W = 4 wavefronts; the sources j of the tile are split into W * S contiguous chunks,
// one per (wave, grid-y) pair.  Inside a chunk every lane of a wave reads the same source,
// so the source coordinates are wave-uniform: they are fetched with scalar loads into SGPRs
// and used directly as VALU operands, with no LDS traffic and no per-lane address math.
// The W partial sums of a workgroup are combined in LDS in wave order; when the grid is
// split along y (S > 1, used when the targets alone cannot fill 256 CUs), each split
// writes its partial sums to a workspace and lm_finish_kernel adds them in a fixed order.
// Every sum therefore has a fixed order: results are bitwise reproducible run to run.
//
// Epilogues.  The thread that owns target i after the reduction also performs the
// classical RK4 bookkeeping for that particle (stage input for the next stage, the
// k1 + 2k2 + 2k3 running sum, the step update), so a Runge-Kutta stage is one launch
// (two when S > 1) and the state never takes a separate pass through memory.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "lm_internal.h"
#include "lm_math.h"

namespace lm {


// ---------------------------------------------------------------------------------------
// Pair bodies.  `kq` holds the kernel-argument scale in base 2: for the conon
// -log2(e)/sigma, for the Gaussian -log2(e)/sigma^2, so the kernel value is 2^(kq r) or
// 2^(kq r^2) (exp2_nonpos in double, the hardware 2^x in single precision).  The force
// weight's constant (1/sigma for the conon, 2/sigma^2 for the Gaussian) is folded into the
// target momentum `psi` by the caller.  PRE: the positions are in the exponent's units
// (q' = k q with k = -kq for the conon, sqrt(-kq) for the Gaussian), so the kernel value is
// 2^-r' (2^-r'^2) and kq is not used; the conon's weight g/r' times d' is then g d / r, the
// Gaussian's g d' carries a factor k that the caller takes out of psi.
// ---------------------------------------------------------------------------------------

template <int DIM, int KER, bool FORCE, bool PRE = false>
__device__ __forceinline__ void pair_f64(const double (&qi)[DIM], const double (&psi)[DIM],
                                         const double (&qj)[DIM], const double (&pj)[DIM],
                                         double kq, double (&v)[DIM], double (&f)[DIM])
{
    double d[DIM];
    // For the conon the squared distance starts at 1e-300 instead of 0 (an FMA in place of
    // the first multiply, so it costs nothing): for the self pair (d = 0) this gives
    // r ~ 1e-150, g = 1 and a finite w that multiplies d = 0, so the pair adds p_j to v and
    // nothing to f, as the system prescribes; for any other pair s > 1e-284 absorbs it.
    double s = (KER == LM_KERNEL_CONON) ? 1e-300 : 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        d[c] = qi[c] - qj[c];
        s = __builtin_fma(d[c], d[c], s);
    }
    double g, w;
    if constexpr (KER == LM_KERNEL_CONON) {
        const double rho = rsqrt_pos(s);
        const double r = s * rho;
        g = PRE ? exp2_nonpos(-r) : exp2_nonpos(r * kq);
        w = g * rho;
    } else {
        g = PRE ? exp2_nonpos(-s) : exp2_nonpos(s * kq);
        w = g;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) v[c] = __builtin_fma(g, pj[c], v[c]);
    if constexpr (FORCE) {
        double pp = psi[0] * pj[0];
#pragma unroll
        for (int c = 1; c < DIM; ++c) pp = __builtin_fma(psi[c], pj[c], pp);
        const double cw = pp * w;
#pragma unroll
        for (int c = 0; c < DIM; ++c) f[c] = __builtin_fma(cw, d[c], f[c]);
    }
}

template <int DIM, int KER, bool FORCE, bool PRE = false>
__device__ __forceinline__ void pair_f32(const float (&qi)[DIM], const float (&psi)[DIM],
                                         const float (&qj)[DIM], const float (&pj)[DIM],
                                         float kq, float (&v)[DIM], float (&f)[DIM])
{
    float d[DIM];
    float s = (KER == LM_KERNEL_CONON) ? 1e-30f : 0.0f;   // as in pair_f64
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        d[c] = qi[c] - qj[c];
        s = __builtin_fmaf(d[c], d[c], s);
    }
    float g, w;
    if constexpr (KER == LM_KERNEL_CONON) {
        const float rho = rsqrt_f32(s);
        g = PRE ? exp2_f32(-(s * rho)) : exp2_f32(s * rho * kq);
        w = g * rho;
    } else {
        g = PRE ? exp2_f32(-s) : exp2_f32(s * kq);
        w = g;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) v[c] = __builtin_fmaf(g, pj[c], v[c]);
    if constexpr (FORCE) {
        float pp = psi[0] * pj[0];
#pragma unroll
        for (int c = 1; c < DIM; ++c) pp = __builtin_fmaf(psi[c], pj[c], pp);
        const float cw = pp * w;
#pragma unroll
        for (int c = 0; c < DIM; ++c) f[c] = __builtin_fmaf(cw, d[c], f[c]);
    }
}

// ---------------------------------------------------------------------------------------
// Epilogue: what the owner of target i does with its full sums (v, f).
// ---------------------------------------------------------------------------------------

template <class T, int DIM, bool FORCE>
__device__ __forceinline__ void epilogue(const EpiArgs<T>& e, int64_t n, int64_t i,
                                         const double (&v)[DIM], const double (&f)[DIM])
{
    // k = (v + tau p_i, f): the time derivative of particle i at the stage input
    double kq[DIM], kp[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        kq[c] = v[c];
        if (e.tau != 0.0) kq[c] += e.tau * (double)e.in_p[c * n + i];
        kp[c] = FORCE ? f[c] : 0.0;
    }
    switch (e.kind) {
    case EPI_STORE:
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            e.out_q[c * n + i] = (T)kq[c];
            if (FORCE) e.out_p[c * n + i] = (T)kp[c];
        }
        break;
    case EPI_RK1:
    case EPI_RK2:
    case EPI_RK3: {
        // stage s: acc (+)= (1 or 2) k_s ; next stage input = y + a_s dt k_s
        const double a = (e.kind == EPI_RK3) ? e.dt : 0.5 * e.dt;
        const double wgt = (e.kind == EPI_RK1) ? 1.0 : 2.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t k = c * n + i;
            double aq = wgt * kq[c];
            if (e.kind != EPI_RK1) aq += (double)e.acc_q[k];
            e.acc_q[k] = (T)aq;
            const double nq = (double)e.base_q[k] + a * kq[c];
            e.out_q[k] = (T)(e.qscale > 0.0 ? e.qscale * nq : nq);
            if constexpr (FORCE) {
                // (without forces the targets are passive points: positions only)
                double ap = wgt * kp[c];
                if (e.kind != EPI_RK1) ap += (double)e.acc_p[k];
                e.acc_p[k] = (T)ap;
                e.out_p[k] = (T)((double)e.base_p[k] + a * kp[c]);
            }
        }
        break;
    }
    case EPI_RK4: {
        // y <- y + dt/6 (k1 + 2k2 + 2k3 + k4); out may alias base (own element only)
        const double h6 = e.dt / 6.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t k = c * n + i;
            const double sq = (double)e.acc_q[k] + kq[c];
            const double nq = (double)e.base_q[k] + h6 * sq;
            e.out_q[k] = (T)nq;
            if (e.qscale > 0.0) e.out_qs[k] = (T)(e.qscale * nq);
            if constexpr (FORCE) {
                const double sp = (double)e.acc_p[k] + kp[c];
                e.out_p[k] = (T)((double)e.base_p[k] + h6 * sp);
            }
        }
        break;
    }
    default:
        break;
    }
}

// ---------------------------------------------------------------------------------------
// The pair-sum kernel.
//   grid  = (ceil(nt / 64), S),  block = 64 * kWaves
//   wave w of block (bx, by) sums sources j in [(by*kWaves + w) * jchunk, ... + jchunk)
//   for the targets i = bx*64 + lane.
// Sources: (qs, ps) with ns points; targets: (qt, pt) with nt points (the same arrays for
// the N-particle right-hand side).
// ---------------------------------------------------------------------------------------

// Sums sources [j0, j1) into (v, f) for one target per lane.  Sources are wave-uniform:
// the loads become scalar loads and the values SGPR operands.
template <int DIM, int KER, bool FORCE, bool PRE = false>
__device__ __forceinline__ void sum_sources(const double* __restrict__ qs, const double* __restrict__ ps,
                                            int64_t ns, int64_t j0, int64_t j1, const double (&qi)[DIM],
                                            const double (&psi)[DIM], double kq, double (&v)[DIM],
                                            double (&f)[DIM])
{
    int64_t j = j0;
    for (; j + kUnroll <= j1; j += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            double qj[DIM], pj[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                qj[c] = qs[c * ns + j + u];
                pj[c] = ps[c * ns + j + u];
            }
            pair_f64<DIM, KER, FORCE, PRE>(qi, psi, qj, pj, kq, v, f);
        }
    }
    for (; j < j1; ++j) {
        double qj[DIM], pj[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qj[c] = qs[c * ns + j];
            pj[c] = ps[c * ns + j];
        }
        pair_f64<DIM, KER, FORCE, PRE>(qi, psi, qj, pj, kq, v, f);
    }
}

// Single precision: pairs summed in float over runs of 64 sources, the runs added in double,
// which keeps the rounding error of long sums at the level of one run.
template <int DIM, int KER, bool FORCE, bool PRE = false>
__device__ __forceinline__ void sum_sources(const float* __restrict__ qs, const float* __restrict__ ps,
                                            int64_t ns, int64_t j0, int64_t j1, const float (&qi)[DIM],
                                            const float (&psi)[DIM], double kqd, double (&v)[DIM],
                                            double (&f)[DIM])
{
    const float kq = (float)kqd;
    for (int64_t jr = j0; jr < j1; jr += 64) {
        const int64_t je = (jr + 64 < j1) ? (jr + 64) : j1;
        float vs[DIM], fs[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) { vs[c] = 0.0f; fs[c] = 0.0f; }
        int64_t j = jr;
        for (; j + 4 <= je; j += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float qj[DIM], pj[DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    qj[c] = qs[c * ns + j + u];
                    pj[c] = ps[c * ns + j + u];
                }
                pair_f32<DIM, KER, FORCE, PRE>(qi, psi, qj, pj, kq, vs, fs);
            }
        }
        for (; j < je; ++j) {
            float qj[DIM], pj[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                qj[c] = qs[c * ns + j];
                pj[c] = ps[c * ns + j];
            }
            pair_f32<DIM, KER, FORCE, PRE>(qi, psi, qj, pj, kq, vs, fs);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) { v[c] += (double)vs[c]; f[c] += (double)fs[c]; }
    }
}

// ---------------------------------------------------------------------------------------
// The pair-sum kernel.
//   grid  = (ceil(nt / 64), S),  block = 64 * kWaves
//   wave w of block (bx, by) sums sources j in [(by*kWaves + w) * jchunk, ... + jchunk)
//   for the targets i = bx*64 + lane.
// Sources: (qs, ps) with ns points; targets: (qt, pt) with nt points (the same arrays for
// the N-particle right-hand side).
// CUT: sources are visited tile by tile (64 consecutive sources); a source tile whose
// bounding box lies farther than the cutoff from the target tile's box is skipped as a
// whole -- every pair it holds is farther apart than the cutoff.  The test is wave-uniform,
// so skipping is a scalar branch.
// ---------------------------------------------------------------------------------------

template <class T, int DIM, int KER, bool FORCE, bool CUT, bool PRE = false>
__global__ __launch_bounds__(kTile * kWaves) void lm_pair_kernel(PairArgs<T> a)
{
    const int lane = threadIdx.x & (kTile - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i = (int64_t)blockIdx.x * kTile + lane;
    const bool live = i < a.nt;
    const int64_t ic = live ? i : (a.nt - 1);       // idle lanes read a valid target

    // target data, kept in VGPRs; the force constant is folded into psi
    T qi[DIM], psi[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        qi[c] = PRE ? (T)(a.tscale * (double)a.qt[c * a.nt + ic]) : a.qt[c * a.nt + ic];
        psi[c] = FORCE ? (T)(a.wscale * (double)a.pt[c * a.nt + ic]) : (T)0;
    }

    const int64_t chunk_id = (int64_t)blockIdx.y * kWaves + wave;
    const int64_t j0 = chunk_id * a.jchunk;
    const int64_t j1 = (j0 + a.jchunk < a.ns) ? (j0 + a.jchunk) : a.ns;

    double v[DIM], f[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) { v[c] = 0.0; f[c] = 0.0; }

    if constexpr (!CUT) {
        sum_sources<DIM, KER, FORCE, PRE>(a.qs, a.ps, a.ns, j0, j1, qi, psi, a.kq, v, f);
    } else {
        const double* __restrict__ tb = a.box_t + (int64_t)blockIdx.x * 8;
        double tlo[DIM], thi[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) { tlo[c] = tb[c]; thi[c] = tb[4 + c]; }
        // source tiles are dealt round-robin to the (grid-y, wave) chunks: in a spatial
        // order the tiles near a target tile are consecutive, and dealing them out spreads
        // that work over every wave instead of leaving it to the one whose chunk holds them
        const int64_t ntiles_s = (a.ns + kTile - 1) / kTile;
        const int64_t nchunks = (int64_t)gridDim.y * kWaves;
        for (int64_t t = chunk_id; t < ntiles_s; t += nchunks) {
            const double* __restrict__ sb = a.box_s + t * 8;
            double g2 = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const double gap = __builtin_fmax(__builtin_fmax(sb[c] - thi[c], tlo[c] - sb[4 + c]), 0.0);
                g2 = __builtin_fma(gap, gap, g2);
            }
            if (g2 > a.rc2) continue;
            const int64_t js = t * kTile;
            const int64_t je = (js + kTile < a.ns) ? (js + kTile) : a.ns;
            sum_sources<DIM, KER, FORCE>(a.qs, a.ps, a.ns, js, je, qi, psi, a.kq, v, f);
        }
    }

    // combine the wave partials in wave order
    __shared__ double red[kWaves][2 * DIM][kTile];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        red[wave][c][lane] = v[c];
        red[wave][DIM + c][lane] = f[c];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double sv = red[0][c][lane], sf = red[0][DIM + c][lane];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            sv += red[w][c][lane];
            sf += red[w][DIM + c][lane];
        }
        v[c] = sv;
        f[c] = sf;
    }
    if (!live) return;
    if (gridDim.y > 1) {
        T* part = a.part + (int64_t)blockIdx.y * (2 * DIM) * a.nt;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            part[c * a.nt + i] = (T)v[c];
            part[(DIM + c) * a.nt + i] = (T)f[c];
        }
        return;
    }
    epilogue<T, DIM, FORCE>(a.epi, a.nt, i, v, f);
}

// Adds the partial sums of each target in a fixed order, then runs the epilogue.  A stage
// has only N threads' worth of targets, too few to hide memory latency one thread per target
// (one workgroup per CU at N = 65536), so a workgroup takes 64 targets and its four waves
// split the slots: wave w adds slots w, w + 4, w + 8, ... in increasing order, and wave 0 adds
// the four wave sums in wave order.
// flags (the symmetric kernel with tile skipping, else null): slot s of a target in superblock
// Z (sbp points each) came from superblock pair {Z, s}; a pair flagged 0 wrote nothing there.
// Slots up to which the flagged finish lists the written slots in LDS (beyond: it tests
// every slot's flag as it goes).
constexpr int kFinishListSlots = 2048;

// (At most 128 VGPRs: four workgroups per CU, so the 1024 workgroups of an N = 65536 stage
// run in one round.)
template <class T, int DIM, bool FORCE>
__global__ __launch_bounds__(256, 4) void lm_finish_kernel(const T* __restrict__ part, int nsplit,
                                                        int64_t nt, EpiArgs<T> e, const uint8_t* __restrict__ flags,
                                                        int64_t sbp)
{
    constexpr int NV = FORCE ? 2 * DIM : DIM;
    __shared__ double red[3][NV][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const bool live = i < nt;
    const int64_t slot = (int64_t)(2 * DIM) * nt;
    // the workgroup's 64 targets form one tile, so they share one superblock Z
    const int64_t Z = (int64_t)blockIdx.x * 64 / sbp;
    auto written = [&](int s) -> bool {
        if (flags == nullptr || s >= nsplit - 1 || s == Z) return true;
        const int64_t X = s < Z ? s : Z, Y = s < Z ? Z : s;
        return flags[Y * (Y - 1) / 2 + X] != 0;
    };
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    if (flags == nullptr) {
        // every slot written: a plain strided loop (the compiler keeps the loads in flight;
        // 89 against 94 us per stage at N = 65536 for the explicit four-slot batches below)
        if (live) {
            const T* ps = part + i;
            for (int s = wave; s < nsplit; s += 4)
#pragma unroll
                for (int c = 0; c < NV; ++c) acc[c] += (double)ps[s * slot + c * nt];
        }
    } else if (nsplit <= kFinishListSlots) {
        // with tile skipping most slots hold nothing: the workgroup marks the written slots
        // in a bit mask (one flag per thread), each wave lists its own slots (s = wave mod 4,
        // increasing) in LDS and adds only those, four slots' loads in flight
        __shared__ uint64_t mask[kFinishListSlots / 64];
        __shared__ int list[4][kFinishListSlots / 4];
        for (int base = 0; base < nsplit; base += 256) {
            const int s = base + (int)threadIdx.x;
            const uint64_t b = __ballot(s < nsplit && written(s));
            if (lane == 0) mask[(base >> 6) + wave] = b;
        }
        __syncthreads();
        const uint64_t own = 0x1111111111111111ull << wave;   // bits b with b = wave mod 4
        int cnt = 0;
        for (int k = 0; k < (nsplit + 63) >> 6; ++k) {
            const uint64_t m = mask[k] & own;
            if ((m >> lane) & 1ull) list[wave][cnt + __popcll(m & ((1ull << lane) - 1ull))] = 64 * k + lane;
            cnt += __popcll(m);
        }
        __syncthreads();
        if (live) {
            const T* ps = part + i;
            const int* ls = list[wave];
            int j = 0;
            for (; j + 3 < cnt; j += 4) {
                double x[4][NV];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t s = ls[j + u];
#pragma unroll
                    for (int c = 0; c < NV; ++c) x[u][c] = (double)ps[s * slot + c * nt];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < NV; ++c) acc[c] += x[u][c];
            }
            for (; j < cnt; ++j) {
                const int64_t s = ls[j];
#pragma unroll
                for (int c = 0; c < NV; ++c) acc[c] += (double)ps[s * slot + c * nt];
            }
        }
    } else if (live) {
        // (more slots than the list holds: the partial-sum cap keeps the symmetric plans
        // below it, so this plain loop is a fallback)
        const T* ps = part + i;
        for (int s = wave; s < nsplit; s += 4)
            if (written(s))
#pragma unroll
                for (int c = 0; c < NV; ++c) acc[c] += (double)ps[s * slot + c * nt];
    }
    if (wave > 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) red[wave - 1][c][lane] = acc[c];
    __syncthreads();
    if (wave != 0 || !live) return;
    double v[DIM], f[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        v[c] = acc[c];
        f[c] = FORCE ? acc[DIM + c] : 0.0;
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            v[c] += red[w][c][lane];
            if (FORCE) f[c] += red[w][DIM + c][lane];
        }
    }
    epilogue<T, DIM, FORCE>(e, nt, i, v, f);
}

// ---------------------------------------------------------------------------------------
// Reductions (double precision, fixed order: per-block tree in LDS, then one block adds
// the block results in block order).
// ---------------------------------------------------------------------------------------

constexpr int kRedThreads = 256;

// out[b] = max over this block's elements of |a[k] - b[k]| (float or double inputs, the
// difference taken in double); NaN wins over every number.
template <class TA, class TB>
__global__ __launch_bounds__(kRedThreads) void lm_maxabsdiff_kernel(const TA* __restrict__ x,
                                                                    const TB* __restrict__ y,
                                                                    int64_t m, double* __restrict__ out)
{
    __shared__ double sh[kRedThreads];
    double r = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * kRedThreads) {
        const double d = __builtin_fabs((double)x[k] - (double)y[k]);
        r = (d > r || d != d) ? d : r;
    }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double b = sh[threadIdx.x + o], a = sh[threadIdx.x];
            sh[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void lm_max_final_kernel(const double* __restrict__ in, int nb,
                                                                   double* __restrict__ out)
{
    __shared__ double sh[kRedThreads];
    double r = 0.0;
    for (int k = threadIdx.x; k < nb; k += kRedThreads) {
        const double d = in[k];
        r = (d > r || d != d) ? d : r;
    }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double b = sh[threadIdx.x + o], a = sh[threadIdx.x];
            sh[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Per-component dot products: out[(c) * nb + b] = partial of sum_i x[c n + i] y[c n + i]
// over block b's range.  grid = (nb, ncomp).
__global__ __launch_bounds__(kRedThreads) void lm_dot_partial_kernel(const double* __restrict__ x,
                                                                     const double* __restrict__ y,
                                                                     int64_t n, double* __restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const int c = blockIdx.y;
    const double* xc = x + (int64_t)c * n;
    const double* yc = y + (int64_t)c * n;
    double r = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kRedThreads)
        r = __builtin_fma(xc[k], yc[k], r);
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)c * gridDim.x + blockIdx.x] = sh[0];
}

// Sums nb partials per component in block order: out[c] = sum_b in[c nb + b].  One block
// per component.
__global__ __launch_bounds__(kRedThreads) void lm_sum_final_kernel(const double* __restrict__ in, int nb,
                                                                   double* __restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const int c = blockIdx.x;
    double r = 0.0;
    for (int k = threadIdx.x; k < nb; k += kRedThreads) r += in[(int64_t)c * nb + k];
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// ---------------------------------------------------------------------------------------
// Conjugate-gradient vector updates for (K + tau I) x_c = b_c, one system per component.
// The scalars live on the device: rr[c] = r_c.r_c, pap[c] = p_c.A p_c, rr_new[c].
// ---------------------------------------------------------------------------------------

// x += alpha p ; r -= alpha Ap, alpha = rr / pap (per component)
__global__ __launch_bounds__(256) void lm_cg_update_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ ap,
                                                              const double* __restrict__ rr,
                                                              const double* __restrict__ pap, int64_t n)
{
    const int c = blockIdx.y;
    // a component that has converged exactly (p = 0, so p.Ap = 0) stays where it is
    const double alpha = pap[c] > 0.0 ? rr[c] / pap[c] : 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (int64_t)c * n + k;
        x[o] = __builtin_fma(alpha, p[o], x[o]);
        r[o] = __builtin_fma(-alpha, ap[o], r[o]);
    }
}

// p = r + beta p, beta = rr_new / rr (per component)
__global__ __launch_bounds__(256) void lm_cg_update_p_kernel(double* __restrict__ p, const double* __restrict__ r,
                                                             const double* __restrict__ rr_new,
                                                             const double* __restrict__ rr, int64_t n)
{
    const int c = blockIdx.y;
    const double beta = rr[c] > 0.0 ? rr_new[c] / rr[c] : 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (int64_t)c * n + k;
        p[o] = __builtin_fma(beta, p[o], r[o]);
    }
}

// y = x + alpha * z (elementwise, m elements)
__global__ __launch_bounds__(256) void lm_axpy_kernel(double* __restrict__ y, const double* __restrict__ x,
                                                      double alpha, const double* __restrict__ z, int64_t m)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        y[k] = __builtin_fma(alpha, z[k], x[k]);
}

// y[k] = 0
__global__ __launch_bounds__(256) void lm_zero_kernel(double* __restrict__ y, int64_t m)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        y[k] = 0.0;
}

// y[k] = x[k] - z[k]
__global__ __launch_bounds__(256) void lm_sub_kernel(double* __restrict__ y, const double* __restrict__ x,
                                                     const double* __restrict__ z, int64_t m)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        y[k] = x[k] - z[k];
}

// type conversion copy
template <class TO, class TI>
__global__ __launch_bounds__(256) void lm_convert_kernel(TO* __restrict__ y, const TI* __restrict__ x, int64_t m)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        y[k] = (TO)x[k];
}

// ---------------------------------------------------------------------------------------
// Tile bounding boxes and spatial ordering (used by the cutoff mode).
// ---------------------------------------------------------------------------------------

// box[t*8 + c] = min over tile t (64 consecutive points) of coordinate c, box[t*8 + 4 + c] =
// max.  One wavefront per tile; min/max combined across the wave by butterfly shuffles.
template <class T, int DIM>
__global__ __launch_bounds__(256) void lm_tile_box_kernel(const T* __restrict__ q, int64_t n, int64_t ntiles,
                                                          double* __restrict__ box)
{
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= ntiles) return;                     // whole wavefronts leave together
    const int64_t i = t * 64 + lane;
    const int64_t ic = i < n ? i : t * 64;       // tile t holds at least one point
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double lo = (double)q[c * n + ic], hi = lo;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = __builtin_fmin(lo, __shfl_xor(lo, o, 64));
            hi = __builtin_fmax(hi, __shfl_xor(hi, o, 64));
        }
        if (lane == 0) {
            box[t * 8 + c] = lo;
            box[t * 8 + 4 + c] = hi;
        }
    }
}

// Reduces tile boxes to the bounding box of all points: out[c] = min, out[4 + c] = max.
template <int DIM>
__global__ __launch_bounds__(256) void lm_box_union_kernel(const double* __restrict__ box, int64_t ntiles,
                                                           double* __restrict__ out)
{
    __shared__ double sh[2 * DIM][256];
    double lo[DIM], hi[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) { lo[c] = box[c]; hi[c] = box[4 + c]; }
    for (int64_t t = threadIdx.x; t < ntiles; t += 256) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            lo[c] = __builtin_fmin(lo[c], box[t * 8 + c]);
            hi[c] = __builtin_fmax(hi[c], box[t * 8 + 4 + c]);
        }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) { sh[c][threadIdx.x] = lo[c]; sh[DIM + c][threadIdx.x] = hi[c]; }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                sh[c][threadIdx.x] = __builtin_fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + o]);
                sh[DIM + c][threadIdx.x] = __builtin_fmax(sh[DIM + c][threadIdx.x], sh[DIM + c][threadIdx.x + o]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) { out[c] = sh[c][0]; out[4 + c] = sh[DIM + c][0]; }
    }
}

__device__ __forceinline__ uint32_t spread_bits(uint32_t x, int dim)
{
    // insert (dim - 1) zero bits between consecutive bits of x
    uint32_t r = 0;
    const int bits = dim == 2 ? 16 : 10;
    for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1u) << (dim * b);
    return r;
}

// keys[i] = (Morton code of point i in the global box) << 32 | i; padding keys are ~0.
template <class T, int DIM>
__global__ __launch_bounds__(256) void lm_morton_kernel(const T* __restrict__ q, int64_t n, int64_t npad,
                                                        const double* __restrict__ gbox, uint64_t* __restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        keys[i] = ~(uint64_t)0;
        return;
    }
    const uint32_t cells = DIM == 2 ? 65536u : 1024u;
    uint32_t code = 0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double lo = gbox[c], ext = gbox[4 + c] - gbox[c];
        double u = ext > 0.0 ? ((double)q[c * n + i] - lo) / ext : 0.0;
        u = __builtin_fmin(__builtin_fmax(u, 0.0), 1.0);
        uint32_t cell = (uint32_t)(u * (double)cells);
        if (cell >= cells) cell = cells - 1;
        code |= spread_bits(cell, DIM) << c;
    }
    keys[i] = ((uint64_t)code << 32) | (uint64_t)i;
}

// Bitonic sort of npad (a power of two) 64-bit keys, ascending.
// lm_bitonic_tile_kernel sorts/merges within tiles of kSortTile keys held in LDS;
// lm_bitonic_step_kernel does one compare-exchange step with partner distance j >= kSortTile.
constexpr int kSortTile = 1024;

__device__ __forceinline__ void cmp_swap(uint64_t& a, uint64_t& b, bool up)
{
    if ((a > b) == up) {
        const uint64_t t = a;
        a = b;
        b = t;
    }
}

// k_lo == 0: full sort of each tile (k = 2 .. tile); else the merge steps j = tile/2 .. 1
// of bitonic stage k = k_lo (> tile).
__global__ __launch_bounds__(kSortTile / 2) void lm_bitonic_tile_kernel(uint64_t* __restrict__ keys, int64_t npad,
                                                                         int64_t k_lo)
{
    __shared__ uint64_t sh[kSortTile];
    const int tile = (int)(npad < kSortTile ? npad : kSortTile);
    const int64_t base = (int64_t)blockIdx.x * tile;
    for (int e = threadIdx.x; e < tile; e += blockDim.x) sh[e] = keys[base + e];
    __syncthreads();
    const int half = tile / 2;
    if (k_lo == 0) {
        for (int k = 2; k <= tile; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int pidx = threadIdx.x; pidx < half; pidx += blockDim.x) {
                    const int li = 2 * j * (pidx / j) + (pidx % j);
                    const bool up = (((base + li) & k) == 0);
                    cmp_swap(sh[li], sh[li + j], up);
                }
                __syncthreads();
            }
        }
    } else {
        for (int j = tile >> 1; j > 0; j >>= 1) {
            for (int pidx = threadIdx.x; pidx < half; pidx += blockDim.x) {
                const int li = 2 * j * (pidx / j) + (pidx % j);
                const bool up = (((base + li) & k_lo) == 0);
                cmp_swap(sh[li], sh[li + j], up);
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < tile; e += blockDim.x) keys[base + e] = sh[e];
}

__global__ __launch_bounds__(256) void lm_bitonic_step_kernel(uint64_t* __restrict__ keys, int64_t npad, int64_t k,
                                                              int64_t j)
{
    const int64_t pidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pidx >= npad / 2) return;
    const int64_t i = 2 * j * (pidx / j) + (pidx % j);
    uint64_t a = keys[i], b = keys[i + j];
    cmp_swap(a, b, (i & k) == 0);
    keys[i] = a;
    keys[i + j] = b;
}

__global__ __launch_bounds__(256) void lm_perm_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                      int64_t* __restrict__ perm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (int64_t)(keys[i] & 0xffffffffull);
}

// out[c][i] = in[c][perm[i]]  (gather)  or  out[c][perm[i]] = in[c][i]  (scatter)
template <class TO, class TI, bool SCATTER>
__global__ __launch_bounds__(256) void lm_permute_kernel(TO* __restrict__ out, const TI* __restrict__ in,
                                                         const int64_t* __restrict__ perm, int64_t n, int dim)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t pi = perm[i];
    for (int c = 0; c < dim; ++c) {
        if (SCATTER)
            out[c * n + pi] = (TO)in[c * n + i];
        else
            out[c * n + i] = (TO)in[c * n + pi];
    }
}

// ---------------------------------------------------------------------------------------
// Launchers (host side).
// ---------------------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t m, int threads, unsigned cap = 8192)
{
    int64_t b = (m + threads - 1) / threads;
    if (b < 1) b = 1;
    return (unsigned)(b < (int64_t)cap ? b : cap);
}

template <class T, int DIM, int KER, bool FORCE, bool CUT>
static hipError_t launch_pair_t(const PairArgs<T>& a, const PairPlan& pl, hipStream_t st)
{
    hipError_t err;
    uint8_t* flags = nullptr;   // symmetric with tile skipping: which superblock pairs wrote
    int64_t sbp = kTile;
    if (pl.sym_waves > 0) {
        if (a.tscale > 0.0) return hipErrorInvalidValue;   // the symmetric kernels scale positions themselves
        {
            SymArgs<T> s{};
            s.q = a.qs;
            s.p = a.ps;
            s.n = a.nt;
            s.nsb = pl.sym_nsb;
            s.rows = pl.sym_rows;
            s.kq = a.kq;
            s.wscale = a.wscale;
            s.part = a.part;
            if (CUT) {
                if (a.box_t != a.box_s) return hipErrorInvalidValue;   // one point set
                s.box = a.box_s;
                s.rc2 = a.rc2;
                s.flags = (uint8_t*)(a.part + (int64_t)pl.nsplit * (2 * DIM) * a.nt);
                flags = s.flags;
                sbp = (int64_t)kTile * pl.sym_rows * pl.sym_waves;
            }
            err = launch_sym_pair<T>(DIM, KER, FORCE, s, pl.sym_waves, st);
        }
    } else {
        dim3 grid((unsigned)pl.itiles, (unsigned)pl.nsplit);
        if (a.tscale > 0.0) {
            if constexpr (CUT) return hipErrorInvalidValue;   // boxes and cutoff are in the original units
            else hipLaunchKernelGGL((lm_pair_kernel<T, DIM, KER, FORCE, false, true>), grid, dim3(kTile * kWaves), 0, st, a);
        } else {
            hipLaunchKernelGGL((lm_pair_kernel<T, DIM, KER, FORCE, CUT>), grid, dim3(kTile * kWaves), 0, st, a);
        }
        err = hipGetLastError();
    }
    if (err != hipSuccess || pl.nsplit == 1) return err;
    hipLaunchKernelGGL((lm_finish_kernel<T, DIM, FORCE>), dim3(blocks_for(a.nt, 64, 1u << 30)), dim3(256), 0, st,
                       (const T*)a.part, pl.nsplit, a.nt, a.epi, (const uint8_t*)flags, sbp);
    return hipGetLastError();
}

template <class T, int DIM, int KER>
static hipError_t launch_pair_k(bool force, bool cut, const PairArgs<T>& a, const PairPlan& pl, hipStream_t st)
{
    if (force) return cut ? launch_pair_t<T, DIM, KER, true, true>(a, pl, st)
                          : launch_pair_t<T, DIM, KER, true, false>(a, pl, st);
    return cut ? launch_pair_t<T, DIM, KER, false, true>(a, pl, st)
               : launch_pair_t<T, DIM, KER, false, false>(a, pl, st);
}

template <class T>
hipError_t launch_pair(int dim, int kernel, bool force, const PairArgs<T>& a, const PairPlan& pl,
                       hipStream_t st)
{
    const bool cut = a.box_s != nullptr;
    if (dim == 2)
        return kernel == LM_KERNEL_CONON ? launch_pair_k<T, 2, LM_KERNEL_CONON>(force, cut, a, pl, st)
                                         : launch_pair_k<T, 2, LM_KERNEL_GAUSS>(force, cut, a, pl, st);
    return kernel == LM_KERNEL_CONON ? launch_pair_k<T, 3, LM_KERNEL_CONON>(force, cut, a, pl, st)
                                     : launch_pair_k<T, 3, LM_KERNEL_GAUSS>(force, cut, a, pl, st);
}

template hipError_t launch_pair<double>(int, int, bool, const PairArgs<double>&, const PairPlan&, hipStream_t);
template hipError_t launch_pair<float>(int, int, bool, const PairArgs<float>&, const PairPlan&, hipStream_t);

int reduce_blocks(int64_t m) { return (int)blocks_for(m, kRedThreads, 1024); }

template <class TA, class TB>
hipError_t launch_maxabsdiff(const TA* x, const TB* y, int64_t m, double* partial, double* out, hipStream_t st)
{
    const int nb = reduce_blocks(m);
    hipLaunchKernelGGL((lm_maxabsdiff_kernel<TA, TB>), dim3(nb), dim3(kRedThreads), 0, st, x, y, m, partial);
    hipLaunchKernelGGL(lm_max_final_kernel, dim3(1), dim3(kRedThreads), 0, st, (const double*)partial, nb, out);
    return hipGetLastError();
}

template hipError_t launch_maxabsdiff<double, double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template hipError_t launch_maxabsdiff<double, float>(const double*, const float*, int64_t, double*, double*, hipStream_t);

hipError_t launch_dots(const double* x, const double* y, int64_t n, int ncomp, double* partial, double* out,
                       hipStream_t st)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(lm_dot_partial_kernel, dim3(nb, ncomp), dim3(kRedThreads), 0, st, x, y, n, partial);
    hipLaunchKernelGGL(lm_sum_final_kernel, dim3(ncomp), dim3(kRedThreads), 0, st, (const double*)partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_cg_update_xr(double* x, double* r, const double* p, const double* ap, const double* rr,
                               const double* pap, int64_t n, int ncomp, hipStream_t st)
{
    hipLaunchKernelGGL(lm_cg_update_xr_kernel, dim3(blocks_for(n, 256, 2048), ncomp), dim3(256), 0, st,
                       x, r, p, ap, rr, pap, n);
    return hipGetLastError();
}

hipError_t launch_cg_update_p(double* p, const double* r, const double* rr_new, const double* rr, int64_t n,
                              int ncomp, hipStream_t st)
{
    hipLaunchKernelGGL(lm_cg_update_p_kernel, dim3(blocks_for(n, 256, 2048), ncomp), dim3(256), 0, st,
                       p, r, rr_new, rr, n);
    return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double alpha, const double* z, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(lm_axpy_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, y, x, alpha, z, m);
    return hipGetLastError();
}

hipError_t launch_zero(double* y, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(lm_zero_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, y, m);
    return hipGetLastError();
}

hipError_t launch_sub(double* y, const double* x, const double* z, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(lm_sub_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, y, x, z, m);
    return hipGetLastError();
}

template <class TO, class TI>
hipError_t launch_convert(TO* y, const TI* x, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL((lm_convert_kernel<TO, TI>), dim3(blocks_for(m, 256)), dim3(256), 0, st, y, x, m);
    return hipGetLastError();
}

template hipError_t launch_convert<float, double>(float*, const double*, int64_t, hipStream_t);

template <class T>
__global__ __launch_bounds__(256) void lm_scaled_copy_kernel(T* __restrict__ y, const T* __restrict__ x, double alpha,
                                                             int64_t m)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
        y[k] = (T)(alpha * (double)x[k]);
}

template <class T>
hipError_t launch_scaled_copy(T* y, const T* x, double alpha, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(lm_scaled_copy_kernel<T>, dim3(blocks_for(m, 256)), dim3(256), 0, st, y, x, alpha, m);
    return hipGetLastError();
}
template hipError_t launch_scaled_copy<float>(float*, const float*, double, int64_t, hipStream_t);
template hipError_t launch_scaled_copy<double>(double*, const double*, double, int64_t, hipStream_t);

int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

template <class T>
hipError_t launch_tile_boxes(int dim, const T* q, int64_t n, double* box, hipStream_t st)
{
    const int64_t nt = tiles_of(n);
    const unsigned g = (unsigned)((nt + 3) / 4);
    if (dim == 2)
        hipLaunchKernelGGL((lm_tile_box_kernel<T, 2>), dim3(g), dim3(256), 0, st, q, n, nt, box);
    else
        hipLaunchKernelGGL((lm_tile_box_kernel<T, 3>), dim3(g), dim3(256), 0, st, q, n, nt, box);
    return hipGetLastError();
}

template hipError_t launch_tile_boxes<double>(int, const double*, int64_t, double*, hipStream_t);
template hipError_t launch_tile_boxes<float>(int, const float*, int64_t, double*, hipStream_t);

int64_t sort_pad(int64_t n)
{
    int64_t p = 2;
    while (p < n) p <<= 1;
    return p;
}

template <class T>
hipError_t launch_morton_order(int dim, const T* q, int64_t n, double* box, double* gbox, uint64_t* keys,
                               int64_t* perm, hipStream_t st)
{
    hipError_t e = launch_tile_boxes<T>(dim, q, n, box, st);
    if (e != hipSuccess) return e;
    const int64_t nt = tiles_of(n);
    if (dim == 2)
        hipLaunchKernelGGL((lm_box_union_kernel<2>), dim3(1), dim3(256), 0, st, (const double*)box, nt, gbox);
    else
        hipLaunchKernelGGL((lm_box_union_kernel<3>), dim3(1), dim3(256), 0, st, (const double*)box, nt, gbox);
    const int64_t npad = sort_pad(n);
    const unsigned gk = (unsigned)((npad + 255) / 256);
    if (dim == 2)
        hipLaunchKernelGGL((lm_morton_kernel<T, 2>), dim3(gk), dim3(256), 0, st, q, n, npad, (const double*)gbox, keys);
    else
        hipLaunchKernelGGL((lm_morton_kernel<T, 3>), dim3(gk), dim3(256), 0, st, q, n, npad, (const double*)gbox, keys);
    const int64_t tile = npad < kSortTile ? npad : kSortTile;
    hipLaunchKernelGGL(lm_bitonic_tile_kernel, dim3((unsigned)(npad / tile)), dim3(kSortTile / 2), 0, st, keys, npad,
                       (int64_t)0);
    for (int64_t k = 2 * tile; k <= npad; k <<= 1) {
        for (int64_t j = k >> 1; j >= tile; j >>= 1)
            hipLaunchKernelGGL(lm_bitonic_step_kernel, dim3((unsigned)((npad / 2 + 255) / 256)), dim3(256), 0, st, keys,
                               npad, k, j);
        hipLaunchKernelGGL(lm_bitonic_tile_kernel, dim3((unsigned)(npad / tile)), dim3(kSortTile / 2), 0, st, keys,
                           npad, k);
    }
    hipLaunchKernelGGL(lm_perm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const uint64_t*)keys, n,
                       perm);
    return hipGetLastError();
}

template hipError_t launch_morton_order<double>(int, const double*, int64_t, double*, double*, uint64_t*, int64_t*,
                                                hipStream_t);
template hipError_t launch_morton_order<float>(int, const float*, int64_t, double*, double*, uint64_t*, int64_t*,
                                               hipStream_t);

template <class TO, class TI>
hipError_t launch_permute(TO* out, const TI* in, const int64_t* perm, int64_t n, int dim, bool scatter, hipStream_t st)
{
    const unsigned g = (unsigned)((n + 255) / 256);
    if (scatter)
        hipLaunchKernelGGL((lm_permute_kernel<TO, TI, true>), dim3(g), dim3(256), 0, st, out, in, perm, n, dim);
    else
        hipLaunchKernelGGL((lm_permute_kernel<TO, TI, false>), dim3(g), dim3(256), 0, st, out, in, perm, n, dim);
    return hipGetLastError();
}

template hipError_t launch_permute<double, double>(double*, const double*, const int64_t*, int64_t, int, bool, hipStream_t);
template hipError_t launch_permute<float, float>(float*, const float*, const int64_t*, int64_t, int, bool, hipStream_t);
template hipError_t launch_permute<float, double>(float*, const double*, const int64_t*, int64_t, int, bool, hipStream_t);
template hipError_t launch_permute<double, float>(double*, const float*, const int64_t*, int64_t, int, bool, hipStream_t);
template hipError_t launch_convert<double, float>(double*, const float*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------------------
// Batched pair sums: many independent problems of uneven size, concatenated in one
// component-major array (dim, ntot); problem b owns columns offs[b] .. offs[b+1]-1 and its
// particles interact only with each other.  The work is a list of items, one wavefront
// each: (problem, first target of a 64-target tile, source chunk, chunks of the problem).
// The grid is persistent: every wave walks the list from its global wave id with a stride
// of all waves in the grid.  The host sorts the list by cost (largest first), so the strided
// walk hands every wave a mix of large and small items.  An item whose problem is not split
// (one chunk) runs the epilogue itself; split problems write partial sums that
// lm_batch_finish_kernel adds in chunk order.  Every sum has a fixed order.
// ---------------------------------------------------------------------------------------

template <class T, int DIM, int KER, bool FORCE>
__global__ __launch_bounds__(kTile * kWaves) void lm_batch_pair_kernel(BatchArgs<T> a)
{
    const int lane = threadIdx.x & (kTile - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t stride = (int32_t)gridDim.x * kWaves;
    for (int32_t it = (int32_t)blockIdx.x * kWaves + wave; it < a.nitems; it += stride) {
        const int4 w = a.items[it];
        const int64_t off = a.offs[w.x];
        const int64_t nb = a.offs[w.x + 1] - off;
        const int64_t il = w.y + lane;
        const bool live = il < nb;
        const int64_t ig = off + (live ? il : nb - 1);
        T qi[DIM], psi[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qi[c] = a.q[c * a.ntot + ig];
            psi[c] = FORCE ? (T)(a.wscale * (double)a.p[c * a.ntot + ig]) : (T)0;
        }
        const int64_t chunk = (nb + w.w - 1) / w.w;
        const int64_t j0 = off + (int64_t)w.z * chunk;
        const int64_t j1 = (j0 + chunk < off + nb) ? (j0 + chunk) : (off + nb);
        double v[DIM], f[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) { v[c] = 0.0; f[c] = 0.0; }
        sum_sources<DIM, KER, FORCE>(a.q, a.p, a.ntot, j0, j1, qi, psi, a.kq, v, f);
        if (!live) continue;
        if (w.w == 1) {
            epilogue<T, DIM, FORCE>(a.epi, a.ntot, off + il, v, f);
        } else {
            T* pp = a.part + a.part_off[w.x] + (int64_t)w.z * (2 * DIM) * nb;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                pp[c * nb + il] = (T)v[c];
                pp[(DIM + c) * nb + il] = (T)f[c];
            }
        }
    }
}

// Finish items (problem, first target of a tile, chunks, -): add the chunk partials of each
// target in chunk order and run the epilogue.  Same persistent walk as the pair kernel.
template <class T, int DIM, bool FORCE>
__global__ __launch_bounds__(kTile * kWaves) void lm_batch_finish_kernel(BatchArgs<T> a, const int4* __restrict__ fin,
                                                                        int32_t nfin)
{
    const int lane = threadIdx.x & (kTile - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t stride = (int32_t)gridDim.x * kWaves;
    for (int32_t it = (int32_t)blockIdx.x * kWaves + wave; it < nfin; it += stride) {
        const int4 w = fin[it];
        const int64_t off = a.offs[w.x];
        const int64_t nb = a.offs[w.x + 1] - off;
        const int64_t il = w.y + lane;
        if (il >= nb) continue;
        const T* pp = a.part + a.part_off[w.x];
        double v[DIM], f[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            v[c] = (double)pp[c * nb + il];
            f[c] = (double)pp[(DIM + c) * nb + il];
        }
        for (int s = 1; s < w.z; ++s) {
            const T* ps = pp + (int64_t)s * (2 * DIM) * nb;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                v[c] += (double)ps[c * nb + il];
                f[c] += (double)ps[(DIM + c) * nb + il];
            }
        }
        epilogue<T, DIM, FORCE>(a.epi, a.ntot, off + il, v, f);
    }
}

template <class T, int DIM, int KER>
static hipError_t launch_batch_k(bool force, const BatchArgs<T>& a, const int4* fin, int32_t nfin, int groups,
                                 hipStream_t st)
{
    const dim3 blk(kTile * kWaves);
    if (a.nitems > 0) {
        if (force)
            hipLaunchKernelGGL((lm_batch_pair_kernel<T, DIM, KER, true>), dim3(groups), blk, 0, st, a);
        else
            hipLaunchKernelGGL((lm_batch_pair_kernel<T, DIM, KER, false>), dim3(groups), blk, 0, st, a);
    }
    if (a.nsym > 0) {
        const hipError_t err = launch_batch_sym<T>(DIM, KER, force, a, st);
        if (err != hipSuccess) return err;
    }
    if (nfin > 0) {
        const int fg = (int)((nfin + kWaves - 1) / kWaves);
        const int cap = groups > 1024 ? groups : 1024;
        const int g = fg < cap ? fg : cap;
        if (force)
            hipLaunchKernelGGL((lm_batch_finish_kernel<T, DIM, true>), dim3(g), blk, 0, st, a, fin, nfin);
        else
            hipLaunchKernelGGL((lm_batch_finish_kernel<T, DIM, false>), dim3(g), blk, 0, st, a, fin, nfin);
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_batch_pair(int dim, int kernel, bool force, const BatchArgs<T>& a, const int4* fin, int32_t nfin,
                             int groups, hipStream_t st)
{
    if (dim == 2)
        return kernel == LM_KERNEL_CONON ? launch_batch_k<T, 2, LM_KERNEL_CONON>(force, a, fin, nfin, groups, st)
                                         : launch_batch_k<T, 2, LM_KERNEL_GAUSS>(force, a, fin, nfin, groups, st);
    return kernel == LM_KERNEL_CONON ? launch_batch_k<T, 3, LM_KERNEL_CONON>(force, a, fin, nfin, groups, st)
                                     : launch_batch_k<T, 3, LM_KERNEL_GAUSS>(force, a, fin, nfin, groups, st);
}
template hipError_t launch_batch_pair<double>(int, int, bool, const BatchArgs<double>&, const int4*, int32_t, int,
                                              hipStream_t);
template hipError_t launch_batch_pair<float>(int, int, bool, const BatchArgs<float>&, const int4*, int32_t, int,
                                             hipStream_t);

// Per-problem reductions over the concatenated layout, one workgroup per problem, in a
// fixed order (strided partial per thread, then a tree in LDS).
//   max:  out[b] = max over c, i of |x[c][i] - y[c][i]|   (NaN wins)
//   dot:  out[b] = sum over c, i of x[c][i] * y[c][i]
template <class TX, bool MAX>
__global__ __launch_bounds__(kRedThreads) void lm_batch_reduce_kernel(const TX* __restrict__ x,
                                                                      const double* __restrict__ y, int dim,
                                                                      int64_t ntot, const int64_t* __restrict__ offs,
                                                                      double* __restrict__ out)
{
    __shared__ double sh[kRedThreads];
    const int64_t off = offs[blockIdx.x], nb = offs[blockIdx.x + 1] - off;
    double r = 0.0;
    for (int c = 0; c < dim; ++c)
        for (int64_t i = threadIdx.x; i < nb; i += kRedThreads) {
            const int64_t k = c * ntot + off + i;
            if (MAX) {
                const double d = __builtin_fabs((double)x[k] - y[k]);
                r = (d > r || d != d) ? d : r;
            } else {
                r = __builtin_fma((double)x[k], y[k], r);
            }
        }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double b = sh[threadIdx.x + o], av = sh[threadIdx.x];
            sh[threadIdx.x] = MAX ? ((b > av || b != b) ? b : av) : av + b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

template <class TX>
hipError_t launch_batch_maxabsdiff(const TX* x, const double* y, int dim, int64_t ntot, const int64_t* offs, int nprob,
                                   double* out, hipStream_t st)
{
    hipLaunchKernelGGL((lm_batch_reduce_kernel<TX, true>), dim3(nprob), dim3(kRedThreads), 0, st, x, y, dim, ntot, offs,
                       out);
    return hipGetLastError();
}
template hipError_t launch_batch_maxabsdiff<double>(const double*, const double*, int, int64_t, const int64_t*, int,
                                                    double*, hipStream_t);
template hipError_t launch_batch_maxabsdiff<float>(const float*, const double*, int, int64_t, const int64_t*, int,
                                                   double*, hipStream_t);

hipError_t launch_batch_dot(const double* x, const double* y, int dim, int64_t ntot, const int64_t* offs, int nprob,
                            double* out, hipStream_t st)
{
    hipLaunchKernelGGL((lm_batch_reduce_kernel<double, false>), dim3(nprob), dim3(kRedThreads), 0, st, x, y, dim, ntot,
                       offs, out);
    return hipGetLastError();
}

// p[c][i] += h * x[c][i] for the particles of problems whose flag is set (one workgroup per
// problem).
__global__ __launch_bounds__(256) void lm_batch_axpy_kernel(double* __restrict__ p, const double* __restrict__ x,
                                                            double h, int dim, int64_t ntot,
                                                            const int64_t* __restrict__ offs,
                                                            const int* __restrict__ active)
{
    if (!active[blockIdx.x]) return;
    const int64_t off = offs[blockIdx.x], nb = offs[blockIdx.x + 1] - off;
    for (int c = 0; c < dim; ++c)
        for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
            const int64_t k = c * ntot + off + i;
            p[k] = __builtin_fma(h, x[k], p[k]);
        }
}

hipError_t launch_batch_axpy(double* p, const double* x, double h, int dim, int64_t ntot, const int64_t* offs,
                             const int* active, int nprob, hipStream_t st)
{
    hipLaunchKernelGGL(lm_batch_axpy_kernel, dim3(nprob), dim3(256), 0, st, p, x, h, dim, ntot, offs, active);
    return hipGetLastError();
}

// dst[c][i] = src[c][i] (with type conversion) for the particles of flagged problems.
template <class TO, class TI>
__global__ __launch_bounds__(256) void lm_batch_copy_kernel(TO* __restrict__ dst, const TI* __restrict__ src, int dim,
                                                            int64_t ntot, const int64_t* __restrict__ offs,
                                                            const int* __restrict__ flag)
{
    if (!flag[blockIdx.x]) return;
    const int64_t off = offs[blockIdx.x], nb = offs[blockIdx.x + 1] - off;
    for (int c = 0; c < dim; ++c)
        for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) dst[c * ntot + off + i] = (TO)src[c * ntot + off + i];
}

hipError_t launch_batch_copy_f32_to_f64(double* dst, const float* src, int dim, int64_t ntot, const int64_t* offs,
                                        const int* flag, int nprob, hipStream_t st)
{
    hipLaunchKernelGGL((lm_batch_copy_kernel<double, float>), dim3(nprob), dim3(256), 0, st, dst, src, dim, ntot, offs,
                       flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Whole shoots of small problems in one launch.  A problem of at most kSmallMax points fits
// one workgroup: its stage input lives in LDS, each owner thread keeps its particle's RK4
// state (step input and running sum, in double precision) in registers, and all
// 4 x steps stages run inside the kernel with two barriers each.  This removes the one
// launch per stage that bounds small problems by launch latency.  The W waves split the work
// as (target tile, source chunk): one tile and W chunks up to 64 points, two tiles and W/2
// chunks up to 128, four tiles and W/4 chunks beyond; chunk partials are added in chunk
// order.  W = 4 up to 64 points (32 in single precision), 8 beyond: more waves hide the
// dependency latency that one wave per SIMD leaves exposed, once each wave has enough pairs to
// pay for the longer barriers and sums (100 RK4 steps, ms, W = 4 / 8 / 16: FP64 2-D 64 points
// 1.06 / 1.07 / 1.13, 96 points 2.55 / 2.16 / 2.18; FP32 2-D 64 points 0.75 / 0.69 / 0.90).
// Shoots take this path up to 128 points (small_path).  One workgroup per problem: grid =
// problems (offs non-null) or one problem of ntot points.
// ---------------------------------------------------------------------------------------

template <int DIM, int KER>
__device__ __forceinline__ void sum_lds(const double* __restrict__ sq, const double* __restrict__ sp, int j0, int j1,
                                        const double (&qi)[DIM], const double (&psi)[DIM], double kq,
                                        double (&v)[DIM], double (&f)[DIM])
{
    for (int j = j0; j < j1; ++j) {
        double qj[DIM], pj[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qj[c] = sq[c * kSmallMax + j];
            pj[c] = sp[c * kSmallMax + j];
        }
        pair_f64<DIM, KER, true>(qi, psi, qj, pj, kq, v, f);
    }
}

// single precision: the chunk (at most 64 sources) is one run summed in float
template <int DIM, int KER>
__device__ __forceinline__ void sum_lds(const float* __restrict__ sq, const float* __restrict__ sp, int j0, int j1,
                                        const float (&qi)[DIM], const float (&psi)[DIM], double kqd,
                                        double (&v)[DIM], double (&f)[DIM])
{
    const float kq = (float)kqd;
    float vs[DIM], fs[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) { vs[c] = 0.0f; fs[c] = 0.0f; }
    for (int j = j0; j < j1; ++j) {
        float qj[DIM], pj[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qj[c] = sq[c * kSmallMax + j];
            pj[c] = sp[c * kSmallMax + j];
        }
        pair_f32<DIM, KER, true>(qi, psi, qj, pj, kq, vs, fs);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) { v[c] += (double)vs[c]; f[c] += (double)fs[c]; }
}

template <class T, int DIM, int KER, int W>
__global__ __launch_bounds__(64 * W) void lm_small_shoot_kernel(SmallShootArgs<T> a)
{
    __shared__ T sq[DIM * kSmallMax];
    __shared__ T sp[DIM * kSmallMax];
    __shared__ double red[W][2 * DIM][64];    // each wave's partials, by lane
    const int64_t off = a.offs ? a.offs[blockIdx.x] : 0;
    const int n = a.offs ? (int)(a.offs[blockIdx.x + 1] - off) : (int)a.ntot;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles = (n + 63) / 64;
    const int tp = tiles <= 1 ? 1 : (tiles <= 2 ? 2 : 4);
    const int nchunk = W / tp;
    const int tile = wave % tp, chunk = wave / tp;
    const int i = tile * 64 + lane;
    const int ic = i < n ? i : n - 1;
    const bool owner = chunk == 0 && i < n;
    const int clen = (n + nchunk - 1) / nchunk;
    const int j0 = chunk * clen < n ? chunk * clen : n;
    const int j1 = j0 + clen < n ? j0 + clen : n;

    for (int e = threadIdx.x; e < n; e += blockDim.x)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            sq[c * kSmallMax + e] = a.q[c * a.ntot + off + e];
            sp[c * kSmallMax + e] = a.p[c * a.ntot + off + e];
        }
    double yq[DIM], yp[DIM], cq[DIM], cp[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        yq[c] = owner ? (double)a.q[c * a.ntot + off + i] : 0.0;
        yp[c] = owner ? (double)a.p[c * a.ntot + off + i] : 0.0;
        cq[c] = 0.0;
        cp[c] = 0.0;
    }
    __syncthreads();

    for (int s = 0; s < a.steps; ++s) {
        for (int k = 0; k < 4; ++k) {
            T qi[DIM], psi[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                qi[c] = sq[c * kSmallMax + ic];
                psi[c] = (T)(a.wscale * (double)sp[c * kSmallMax + ic]);
            }
            double v[DIM], f[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) { v[c] = 0.0; f[c] = 0.0; }
            sum_lds<DIM, KER>(sq, sp, j0, j1, qi, psi, a.kq, v, f);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                red[wave][c][lane] = v[c];
                red[wave][DIM + c][lane] = f[c];
            }
            __syncthreads();
            if (owner) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    // chunk ch of this tile is wave ch * tp + tile (the owner's wave is chunk 0)
                    double sv = red[tile][c][lane], sf = red[tile][DIM + c][lane];
                    for (int ch = 1; ch < nchunk; ++ch) {
                        sv += red[ch * tp + tile][c][lane];
                        sf += red[ch * tp + tile][DIM + c][lane];
                    }
                    const double kqc = sv + a.tau * (double)sp[c * kSmallMax + i];
                    const double kpc = sf;
                    double nq, np;
                    if (k == 0) {
                        cq[c] = kqc;
                        cp[c] = kpc;
                        nq = yq[c] + 0.5 * a.dt * kqc;
                        np = yp[c] + 0.5 * a.dt * kpc;
                    } else if (k < 3) {
                        cq[c] += 2.0 * kqc;
                        cp[c] += 2.0 * kpc;
                        const double h = (k == 2) ? a.dt : 0.5 * a.dt;
                        nq = yq[c] + h * kqc;
                        np = yp[c] + h * kpc;
                    } else {
                        const double h6 = a.dt / 6.0;
                        yq[c] = yq[c] + h6 * (cq[c] + kqc);
                        yp[c] = yp[c] + h6 * (cp[c] + kpc);
                        nq = yq[c];
                        np = yp[c];
                    }
                    sq[c * kSmallMax + i] = (T)nq;
                    sp[c * kSmallMax + i] = (T)np;
                }
            }
            __syncthreads();
        }
    }
    if (owner)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            a.q[c * a.ntot + off + i] = (T)yq[c];
            a.p[c * a.ntot + off + i] = (T)yp[c];
        }
}

template <class T, int DIM, int KER>
hipError_t launch_small_shoot_w(const SmallShootArgs<T>& a, int problems, int waves, hipStream_t st)
{
    if (waves == 4)
        hipLaunchKernelGGL((lm_small_shoot_kernel<T, DIM, KER, 4>), dim3(problems), dim3(256), 0, st, a);
    else if (waves == 8)
        hipLaunchKernelGGL((lm_small_shoot_kernel<T, DIM, KER, 8>), dim3(problems), dim3(512), 0, st, a);
    else
        hipLaunchKernelGGL((lm_small_shoot_kernel<T, DIM, KER, 16>), dim3(problems), dim3(1024), 0, st, a);
    return hipGetLastError();
}

static int small_shoot_waves(int64_t n, bool fp32)
{
    // LM_SMALL_WAVES = 4, 8 or 16 fixes the width (tuning and tests; read at every launch)
    const char* e = getenv("LM_SMALL_WAVES");
    const int fixed = e ? atoi(e) : 0;
    if (fixed == 4 || fixed == 8 || fixed == 16) return fixed;
    return n <= (fp32 ? 32 : 64) ? 4 : (n <= 128 ? 8 : 16);   // 16: only under LM_SMALL = 1
}

// Measured (100 RK4 steps, ms; one workgroup of 4 / 8 / 16 waves against one launch per stage):
// FP64 2-D 96 points 2.55 / 2.16 / 2.18 against 2.46, 128 points 3.33 / 2.77 / 2.74 against 2.96,
// 160 points 7.99 / 6.40 / 5.99 against 3.37, 256 points 12.67 / 10.10 / 9.40 against 4.64; FP64
// 3-D 128 points 3.96 / 3.20 / 3.25 against 3.55; FP32 2-D 128 points 2.03 / 1.23 / 1.25 against
// 2.16, FP32 3-D 192 points 7.03 / 3.51 / 3.41 against 3.28.  Past two tiles the one-workgroup
// path loses: its work grows as n^2 on one CU while a stage of the other path stays near its
// launch cost.
bool small_path(int64_t n, int dim, bool fp32)
{
    (void)dim;
    (void)fp32;
    const char* e = getenv("LM_SMALL");
    if (e && (e[0] == '0' || e[0] == '1') && e[1] == 0) return e[0] == '1' && n <= kSmallMax;
    return n <= 128;
}

template <class T>
hipError_t launch_small_shoot(int dim, int kernel, const SmallShootArgs<T>& a, int problems, hipStream_t st)
{
    const int w = small_shoot_waves(a.offs ? kSmallMax : a.ntot, sizeof(T) == 4);
    if (dim == 2)
        return kernel == LM_KERNEL_CONON ? launch_small_shoot_w<T, 2, LM_KERNEL_CONON>(a, problems, w, st)
                                         : launch_small_shoot_w<T, 2, LM_KERNEL_GAUSS>(a, problems, w, st);
    return kernel == LM_KERNEL_CONON ? launch_small_shoot_w<T, 3, LM_KERNEL_CONON>(a, problems, w, st)
                                     : launch_small_shoot_w<T, 3, LM_KERNEL_GAUSS>(a, problems, w, st);
}
template hipError_t launch_small_shoot<double>(int, int, const SmallShootArgs<double>&, int, hipStream_t);
template hipError_t launch_small_shoot<float>(int, int, const SmallShootArgs<float>&, int, hipStream_t);

}  // namespace lm
