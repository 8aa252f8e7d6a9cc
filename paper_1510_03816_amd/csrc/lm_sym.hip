// lm_sym.hip -- the N-particle pair sums with each unordered pair evaluated once (gfx950).
//
// In the right-hand side of the N-particle system (equation "N-particle") the kernel value
// G(|q_i - q_j|), the force weight w(|q_i - q_j|) and the momentum product p_i . p_j are
// symmetric in (i, j) and the distance vector q_i - q_j changes sign, so one evaluation of
// a pair serves both particles:
//     v_i += g p_j,  v_j += g p_i,  f_i += (p_i . p_j) w d,  f_j -= (p_i . p_j) w d,  d = q_i - q_j.
// The shared part (distance, 1/sqrt, exponential, weight, momentum product) is about three
// quarters of a pair's work, so a sweep over the N(N+1)/2 unordered pairs costs about 55% of
// the N^2 ordered ones.  Used for the self-interaction of one point set (right-hand side, RK4
// stages, K x, with or without tile skipping, and a batch's larger problems); targets distinct
// from the sources keep the one-sided kernel in lm_kernels.hip.  In single precision a row
// point's pairs with one column tile (64 steps) are summed in float and those sums in double,
// as the one-sided kernel sums runs of 64 sources, and a column point's terms from one wave's
// rows likewise: in float over the tile, in double from there on.
//
// Decomposition.  The 64-point tiles are grouped into superblocks of B = R W tiles; a
// workgroup of W wavefronts takes one pair (X, Y), X <= Y, of superblocks.  Wave w owns the
// R row tiles X*B + R w ... X*B + R w + R - 1 (R = 2, or 4 in the widest tier: one point of
// each per lane, in registers, with their row sums) and the W waves walk the B column tiles
// of superblock Y together:
//   - the column tile (q, p interleaved) is staged in LDS twice in a row, so that at step k
//     lane l reads entry l + k -- point (l + k) mod 64 -- at an immediate offset, and over 64
//     steps every lane meets every point of the tile once;
//   - the column-side terms go to the wave's own LDS array with ds_add_f64 at the same entry
//     l + k (128 entries, the two halves added at the end), so no two lanes of an instruction
//     touch the same word and each wave's sums have a fixed order (single precision: in
//     registers that rotate across the wavefront with the entries, added to the array once
//     per tile);
//   - after the tile, the W waves' arrays are added in wave order and written out.
// In a diagonal superblock (X = Y) a row tile meets the column tiles after it symmetrically,
// itself one-sidedly (all 64 x 64 ordered pairs, the self pair included), and skips the ones
// before it (those pairs are done from the other side).
//
// Partial sums.  A point of superblock Z receives one partial from each superblock pair that
// contains Z: from (Z, Y), Y > Z, as a row (slot Y); from (Y, Z), Y < Z, as a column (slot Y);
// from (Z, Z) both (row: slot Z, column: slot S).  Every one of the S + 1 slots of a point is
// written exactly once per launch (with tile skipping, or flagged empty), and lm_finish_kernel
// adds them in a fixed order, so the result is bitwise reproducible.  The force constant is
// applied when a partial is written.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "lm_internal.h"
#include "lm_math.h"
#include "lm_sym.h"

namespace lm {

namespace {

// Values per staged column point: q and p, padded by one so that the 64 lanes' reads of
// consecutive entries (an odd stride) fall in distinct LDS banks.
__host__ __device__ constexpr int sym_stride(int dim) { return 2 * dim + 1; }

// Words per component of a wave's column array: 128 in double precision (entry l + k at step
// k, the two halves added at the end), 64 in single precision (entry l, written once per tile).
template <class T>
__host__ __device__ constexpr int sym_col_words() { return sizeof(T) == sizeof(double) ? 128 : 64; }

// Dynamic LDS of a workgroup of `waves` wavefronts: their column arrays (EC components) and
// the staged column tile.
template <class T, int DIM>
size_t sym_lds_bytes(int waves, int ec)
{
    return (size_t)waves * ec * sym_col_words<T>() * sizeof(double) + (size_t)128 * sym_stride(DIM) * sizeof(T);
}

__device__ __forceinline__ int64_t tiles_of_dev(int64_t n) { return (n + kSymSteps - 1) / kSymSteps; }

// Per-precision pieces: FMA, the conon's squared-distance floor (see pair_f64), 1/sqrt and the
// exponential 2^x (in single precision the hardware 2^x).
template <class T>
struct SymMath;
template <>
struct SymMath<double> {
    static constexpr double kFloor = 1e-300;
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double rsq(double s) { return rsqrt_pos(s); }
    static __device__ __forceinline__ double ex(double x) { return exp2_nonpos(x); }
};
template <>
struct SymMath<float> {
    static constexpr float kFloor = 1e-30f;
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float rsq(float s) { return rsqrt_f32(s); }
    static __device__ __forceinline__ float ex(float x) { return exp2_f32(x); }
};

// The symmetric part of a pair: d = q_i - q_j, kernel value g and force weight w (without
// the constant, which is applied to the sums).  Positions are in the exponent's units (see
// sym_superblock_pair): the kernel value is 2^-r for the conon, 2^-(r^2) for the Gaussian.
template <class T, int DIM, int KER>
__device__ __forceinline__ void sym_pair(const T (&qi)[DIM], const T (&qj)[DIM], T (&d)[DIM], T& g, T& w)
{
    using M = SymMath<T>;
    // conon: the squared distance starts at a tiny floor so the self pair and padding points
    // at the same position give a finite weight times d = 0
    T s = (KER == LM_KERNEL_CONON) ? M::kFloor : (T)0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        d[c] = qi[c] - qj[c];
        s = M::fma(d[c], d[c], s);
    }
    if constexpr (KER == LM_KERNEL_CONON) {
        const T rho = M::rsq(s);
        g = M::ex(-(s * rho));
        w = g * rho;
    } else {
        g = M::ex(-s);
        w = g;
    }
}

// Lane l receives x of lane (l + 1) mod 64: a rotation of the whole wavefront by one lane
// (DPP wave_rol; every source lane is in range, so bound_ctrl changes nothing and lets the
// compiler fold the move into the add that consumes it).  All 64 lanes must be active: the
// symmetric kernels call it only in code every lane of the wave runs (lanes past n hold zero
// momenta, and every branch around it depends on the wave's tiles alone).
__device__ __forceinline__ float wave_rotate_down(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x134, 0xF, 0xF, true));
}

// One step: the ROWS row points of this lane against column entry cj (q then p).  With
// JSIDE the column-side terms go to the column sums of that entry.  Double precision adds
// them into the wave's column array at `acc` (component c at acc[c * 128]) with ds_add_f64.
// Single precision keeps them in registers, ca[c]: lane l's value is the running sum of the
// entry it meets at this step, and adding the step's terms to the neighbour's value (one
// wavefront rotation, folded into the add) moves every sum along with its entry, since at
// the next step lane l meets the entry lane l + 1 met at this one (the force sums hold +cw d).
template <class T, int DIM, int KER, bool FORCE, int ROWS, bool JSIDE>
__device__ __forceinline__ void sym_step(const T (&qi)[ROWS][DIM], const T (&pi)[ROWS][DIM], const T (&cj)[2 * DIM],
                                         T (&v)[ROWS][DIM], T (&f)[ROWS][DIM], double* __restrict__ acc,
                                         T (&ca)[2 * DIM])
{
    using M = SymMath<T>;
    constexpr bool REG = sizeof(T) == sizeof(float);   // column sums in registers
    T qj[DIM], pj[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        qj[c] = cj[c];
        pj[c] = cj[DIM + c];
    }
    T tv[DIM], tf[DIM];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        T d[DIM], g, w;
        sym_pair<T, DIM, KER>(qi[r], qj, d, g, w);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            v[r][c] = M::fma(g, pj[c], v[r][c]);
            if (JSIDE) tv[c] = (r == 0) ? g * pi[r][c] : M::fma(g, pi[r][c], tv[c]);
        }
        if constexpr (FORCE) {
            T pp = pi[r][0] * pj[0];
#pragma unroll
            for (int c = 1; c < DIM; ++c) pp = M::fma(pi[r][c], pj[c], pp);
            const T cw = pp * w;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                f[r][c] = M::fma(cw, d[c], f[r][c]);
                // the column point's force is -cw d; single precision sums +cw d (FMAs without
                // a negated operand) and subtracts the tile's sum once
                if (JSIDE && REG) tf[c] = (r == 0) ? cw * d[c] : M::fma(cw, d[c], tf[c]);
                if (JSIDE && !REG) tf[c] = (r == 0) ? -cw * d[c] : M::fma(-cw, d[c], tf[c]);
            }
        }
    }
    if constexpr (JSIDE && REG) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            ca[c] = wave_rotate_down(ca[c]) + tv[c];
            if (FORCE) ca[DIM + c] = wave_rotate_down(ca[DIM + c]) + tf[c];
        }
    } else if constexpr (JSIDE) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            __hip_atomic_fetch_add(acc + c * sym_col_words<T>(), (double)tv[c], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            if (FORCE)
                __hip_atomic_fetch_add(acc + (DIM + c) * sym_col_words<T>(), (double)tf[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// All 64 steps of one (row tile(s), column tile) block.  jb = this lane's first column entry
// (jbuf + lane * sym_stride(DIM)), acc = this lane's first word of the wave's column array.
// In single precision the register column sums start at zero; after the 64th step lane l
// holds those of entry l + 63, and one more rotation brings entry l to lane l, which adds
// them (in double) to word l of the column array: each lane owns its word, so no atomics.
template <class T, int DIM, int KER, bool FORCE, int ROWS, bool JSIDE>
__device__ __forceinline__ void sym_block(const T (&qi)[ROWS][DIM], const T (&pi)[ROWS][DIM], const T* __restrict__ jb,
                                          T (&v)[ROWS][DIM], T (&f)[ROWS][DIM], double* __restrict__ acc)
{
    constexpr int E = sym_stride(DIM);
    constexpr bool REG = JSIDE && sizeof(T) == sizeof(float);
    T ca[2 * DIM];
#pragma unroll
    for (int c = 0; c < 2 * DIM; ++c) ca[c] = (T)0;
    if constexpr (sizeof(T) == sizeof(float)) {
        // single precision: the next step's column entry is read while this one is evaluated
        // (after the 64th step that is entry l + 64, the copy of entry l, never used)
        T cj[2 * DIM];
#pragma unroll
        for (int c = 0; c < 2 * DIM; ++c) cj[c] = jb[c];
        for (int k0 = 0; k0 < kSymSteps; k0 += kSymUnroll) {
#pragma unroll
            for (int u = 0; u < kSymUnroll; ++u) {
                T nx[2 * DIM];
#pragma unroll
                for (int c = 0; c < 2 * DIM; ++c) nx[c] = jb[(k0 + u + 1) * E + c];
                sym_step<T, DIM, KER, FORCE, ROWS, JSIDE>(qi, pi, cj, v, f, acc + k0 + u, ca);
#pragma unroll
                for (int c = 0; c < 2 * DIM; ++c) cj[c] = nx[c];
            }
        }
    } else {
        for (int k0 = 0; k0 < kSymSteps; k0 += kSymUnroll) {
#pragma unroll
            for (int u = 0; u < kSymUnroll; ++u) {
                T cj[2 * DIM];
#pragma unroll
                for (int c = 0; c < 2 * DIM; ++c) cj[c] = jb[(k0 + u) * E + c];
                sym_step<T, DIM, KER, FORCE, ROWS, JSIDE>(qi, pi, cj, v, f, acc + k0 + u, ca);
            }
        }
    }
    if constexpr (REG) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            acc[c * sym_col_words<T>()] += (double)wave_rotate_down(ca[c]);
            if (FORCE) acc[(DIM + c) * sym_col_words<T>()] -= (double)wave_rotate_down(ca[DIM + c]);
        }
    }
}

// Loads column tile J into jbuf: entry e (0..127) holds point J*64 + (e mod 64), its q (times
// ks) then its p (the pad word is never read); points past n are zero (zero momentum: they
// add exactly nothing to real points).
template <class T, int DIM>
__device__ __forceinline__ void sym_stage(T* __restrict__ jbuf, const T* __restrict__ q, const T* __restrict__ p,
                                          int64_t ld, int64_t n, int64_t J, T ks)
{
    constexpr int E = sym_stride(DIM);
    for (int t = threadIdx.x; t < kSymSteps * 2 * DIM; t += blockDim.x) {
        const int c = t >> 6, l = t & 63;
        const int64_t j = J * kSymSteps + l;
        T x = (T)0;
        if (j < n) x = (c < DIM) ? ks * q[c * ld + j] : p[(c - DIM) * ld + j];
        jbuf[l * E + c] = x;
        jbuf[(l + 64) * E + c] = x;
    }
}

// The same in two halves, so that the global reads of the next tile can be issued before the
// current one is evaluated: sym_fetch reads this thread's values into registers, sym_put
// stores them.  For workgroups where kSymFetch values per thread cover the tile
// (sym_fetch_fits); narrower ones stage with sym_stage.
constexpr int kSymFetch = 2;
template <int DIM>
__device__ __forceinline__ bool sym_fetch_fits()
{
    return (int)blockDim.x * kSymFetch >= kSymSteps * 2 * DIM;
}
template <class T, int DIM>
__device__ __forceinline__ void sym_fetch(T (&x)[kSymFetch], const T* __restrict__ q, const T* __restrict__ p,
                                          int64_t ld, int64_t n, int64_t J, T ks)
{
#pragma unroll
    for (int u = 0; u < kSymFetch; ++u) {
        const int t = threadIdx.x + u * blockDim.x;
        const int c = t >> 6, l = t & 63;
        const int64_t j = J * kSymSteps + l;
        x[u] = (T)0;
        if (t < kSymSteps * 2 * DIM && j < n) x[u] = (c < DIM) ? ks * q[c * ld + j] : p[(c - DIM) * ld + j];
    }
}
template <class T, int DIM>
__device__ __forceinline__ void sym_put(T* __restrict__ jbuf, const T (&x)[kSymFetch])
{
    constexpr int E = sym_stride(DIM);
#pragma unroll
    for (int u = 0; u < kSymFetch; ++u) {
        const int t = threadIdx.x + u * blockDim.x;
        const int c = t >> 6, l = t & 63;
        if (t < kSymSteps * 2 * DIM) {
            jbuf[l * E + c] = x[u];
            jbuf[(l + 64) * E + c] = x[u];
        }
    }
}

// Whether the bounding boxes of tiles a and b (8 doubles each: lo[4], hi[4]) lie farther apart
// than sqrt(rc2), so that every pair between them does.
template <int DIM>
__device__ __forceinline__ bool sym_tiles_far(const double* __restrict__ a, const double* __restrict__ b, double rc2)
{
    double g2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double gap = __builtin_fmax(__builtin_fmax(a[c] - b[4 + c], b[c] - a[4 + c]), 0.0);
        g2 = __builtin_fma(gap, gap, g2);
    }
    return g2 > rc2;
}

// The ROWS row tiles of this wave against column tile J (staged at jb), sums added to (v, f):
// all rows symmetrically in one pass when they allow it, else row by row by mode.  CUT: a row
// tile whose box lies farther than the cutoff from column tile J's box skips it (both
// directions of its pairs: the block is evaluated once, here or nowhere).
template <class T, int DIM, int KER, bool FORCE, bool CUT, int ROWS, class A>
__device__ __forceinline__ void sym_tile(bool diag, const int64_t (&I)[ROWS], int64_t J, int64_t NT,
                                         const T (&qi)[ROWS][DIM], const T (&pi)[ROWS][DIM],
                                         const T* __restrict__ jb, A (&v)[ROWS][DIM], A (&f)[ROWS][DIM],
                                         double* __restrict__ acc, const double* __restrict__ box, double rc2)
{
    bool far[ROWS];
    bool any_far = false;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        far[r] = CUT && I[r] < NT && sym_tiles_far<DIM>(box + I[r] * 8, box + J * 8, rc2);
        any_far = any_far || far[r];
    }
    // every row tile meets J from both sides, except near the diagonal (and skipped tiles)
    const bool all = (diag ? J > I[ROWS - 1] : I[ROWS - 1] < NT) && !any_far;
    if (all) {
        sym_block<T, DIM, KER, FORCE, ROWS, true>(qi, pi, jb, v, f, acc);
        return;
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int m = far[r] ? SYM_SKIP : sym_mode(diag, I[r], J, NT);
        if (m == SYM_SKIP) continue;
        T q1[1][DIM], p1[1][DIM], v1[1][DIM], f1[1][DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            q1[0][c] = qi[r][c];
            p1[0][c] = pi[r][c];
            v1[0][c] = v[r][c];
            f1[0][c] = f[r][c];
        }
        if (m == SYM_BOTH)
            sym_block<T, DIM, KER, FORCE, 1, true>(q1, p1, jb, v1, f1, acc);
        else
            sym_block<T, DIM, KER, FORCE, 1, false>(q1, p1, jb, v1, f1, acc);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            v[r][c] = v1[0][c];
            f[r][c] = f1[0][c];
        }
    }
}

// One workgroup's superblock pair (X, Y) of a point set of n points: component c of point i at
// q[c * ld + i] (ld = n for one problem, the batch's total for a batched one); partial sums in
// part, (S + 1) slots of 2 dim x n values of T (each a double sum, rounded once).  CUT:
// flags[b] (b = the pair's number) says whether the pair wrote its slots; a pair whose tiles
// are all farther apart than the cutoff writes nothing else (lm_finish_kernel skips its slots).
template <class T, int DIM, int KER, bool FORCE, bool CUT, int ROWS>
__device__ __forceinline__ void sym_superblock_pair(const T* __restrict__ q, const T* __restrict__ p, int64_t ld,
                                                    int64_t n, int64_t S, int64_t X, int64_t Y, double kqd,
                                                    double wscale, T* __restrict__ part,
                                                    const double* __restrict__ box, double rc2,
                                                    uint8_t* __restrict__ flags, int64_t b)
{
    constexpr int E = sym_stride(DIM);           // staged values per column point
    constexpr int EC = FORCE ? 2 * DIM : DIM;    // column sums per point
    extern __shared__ double lds_words[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int64_t side = ROWS * (int64_t)nw;
    constexpr int CW = sym_col_words<T>();
    double* region = lds_words;                               // [nw][EC][CW]
    T* jbuf = reinterpret_cast<T*>(region + nw * EC * CW);    // [128][E]

    const bool diag = X == Y;
    const int64_t NT = tiles_of_dev(n);
    // Positions in the exponent's units, q' = ks q: ks = -kq for the conon (the kernel value
    // is then 2^-|q'_i - q'_j|) and sqrt(-kq) for the Gaussian (2^-|q'_i - q'_j|^2), which
    // takes the multiply by kq out of every pair.  The conon's force weight g/r' times d'
    // equals g d / r; the Gaussian's g d' carries one factor ks, divided out of the force
    // constant.  (Tile boxes and the cutoff stay in the original units.)
    const double ksd = (KER == LM_KERNEL_CONON) ? -kqd : __builtin_sqrt(-kqd);
    const T ks = (T)ksd;
    const double fscale = (KER == LM_KERNEL_CONON) ? wscale : wscale / ksd;

    // CUT: bit k of `need` says whether column tile Y * side + k lies within the cutoff of some
    // row tile of the superblock; the others are neither staged nor evaluated (their column
    // sums are written as zeros), and a pair with no such tile writes only its flag
    uint32_t need = ~0u;
    static_assert(!CUT || ROWS <= 2, "with tile skipping a superblock has at most 2 x 16 tiles (one bit each)");
    if constexpr (CUT) {
        __shared__ uint32_t need_bits;
        if (threadIdx.x == 0) need_bits = diag ? ~0u : 0u;
        __syncthreads();
        if (!diag) {
            const int64_t I0 = X * side, I1 = (I0 + side < NT) ? I0 + side : NT;
            const int64_t J0 = Y * side, J1 = (J0 + side < NT) ? J0 + side : NT;
            const int64_t w = J1 - J0;
            uint32_t m = 0;
            for (int64_t t = threadIdx.x; t < (I1 - I0) * w; t += blockDim.x)
                if (!sym_tiles_far<DIM>(box + (I0 + t / w) * 8, box + (J0 + t % w) * 8, rc2)) m |= 1u << (t % w);
            if (m) atomicOr(&need_bits, m);
        }
        __syncthreads();
        need = need_bits;
        if (threadIdx.x == 0) flags[b] = (uint8_t)(need != 0);
        if (need == 0) return;
    }

    // row points in registers; their sums over one column tile in T, over all tiles in double
    int64_t I[ROWS];
    T qi[ROWS][DIM], pi[ROWS][DIM];
    double vs[ROWS][DIM], fs[ROWS][DIM];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        I[r] = X * side + ROWS * wave + r;
        const int64_t i = I[r] * kSymSteps + lane;
        const bool live = i < n;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qi[r][c] = live ? ks * q[c * ld + i] : (T)0;
            pi[r][c] = live ? p[c * ld + i] : (T)0;
            vs[r][c] = 0.0;
            fs[r][c] = 0.0;
        }
    }

    for (int t = threadIdx.x; t < nw * EC * CW; t += blockDim.x) region[t] = 0.0;
    const int64_t J0 = Y * side;
    const int64_t J1 = (J0 + side < NT) ? (J0 + side) : NT;
    if (need & 1u) sym_stage<T, DIM>(jbuf, q, p, ld, n, J0, ks);
    __syncthreads();

    const T* jb = jbuf + lane * E;
    double* acc = region + wave * EC * CW + lane;
    const int64_t slot_col = diag ? S : X;
    T* pc = part + slot_col * (2 * DIM) * n;
    for (int64_t J = J0; J < J1; ++J) {
        // single precision: the next tile's reads are in flight while this one is evaluated
        const bool fetch = sizeof(T) == sizeof(float) && sym_fetch_fits<DIM>();
        const bool next = J + 1 < J1 && ((need >> (J + 1 - J0)) & 1u);
        T nx[kSymFetch];
        if (fetch && next) sym_fetch<T, DIM>(nx, q, p, ld, n, J + 1, ks);
        if constexpr (sizeof(T) == sizeof(double)) {
            sym_tile<T, DIM, KER, FORCE, CUT, ROWS>(diag, I, J, NT, qi, pi, jb, vs, fs, acc, box, rc2);
        } else {
            T v[ROWS][DIM], f[ROWS][DIM];
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    v[r][c] = (T)0;
                    f[r][c] = (T)0;
                }
            sym_tile<T, DIM, KER, FORCE, CUT, ROWS>(diag, I, J, NT, qi, pi, jb, v, f, acc, box, rc2);
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    vs[r][c] += (double)v[r][c];
                    fs[r][c] += (double)f[r][c];
                }
        }
        __syncthreads();
        // column sums of tile J, in double: the waves in order (in double precision each wave's
        // two halves in order)
        for (int t = threadIdx.x; t < EC * 64; t += blockDim.x) {
            const int c = t >> 6, l = t & 63;
            double s = 0.0;
            for (int w = 0; w < nw; ++w) {
                double* rg = region + (w * EC + c) * CW;
                s += rg[l];
                rg[l] = 0.0;
                if (CW == 128) {
                    s += rg[l + 64];
                    rg[l + 64] = 0.0;
                }
            }
            const int64_t j = J * kSymSteps + l;
            if (j < n) pc[c * n + j] = (T)((c < DIM) ? s : s * fscale);
        }
        if (next) {
            if (fetch)
                sym_put<T, DIM>(jbuf, nx);
            else
                sym_stage<T, DIM>(jbuf, q, p, ld, n, J + 1, ks);
        }
        __syncthreads();
    }

    T* pr = part + Y * (2 * DIM) * n;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int64_t i = I[r] * kSymSteps + lane;
        if (I[r] >= NT || i >= n) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            pr[c * n + i] = (T)vs[r][c];
            if (FORCE) pr[(DIM + c) * n + i] = (T)(fs[r][c] * fscale);
        }
    }
}

template <class T, int DIM, int KER, bool FORCE, bool CUT>
__global__ __launch_bounds__(512, kSymOccupancy) void lm_sym_pair_kernel(SymArgs<T> a)
{
    int64_t X, Y;
    sym_superblocks(blockIdx.x, a.nsb, X, Y);
    sym_superblock_pair<T, DIM, KER, FORCE, CUT, kSymRows>(a.q, a.p, a.n, a.n, a.nsb, X, Y, a.kq, a.wscale, a.part,
                                                           a.box, a.rc2, a.flags, blockIdx.x);
}

// The widest tier (double precision with forces, every pair, large N): four row tiles per
// wave, so each staged column entry and each column-array add serves four pairs instead of
// two, at 143-185 VGPRs (three waves per SIMD).  Measured at N = 65536 (two waves per
// workgroup, superblocks of 8 tiles as with two rows and four waves): conon 3613 us per stage
// against 3748, Gaussian 2841 against 2969; at N = 131072 13861 against 14576.
template <class T, int DIM, int KER>
__global__ __launch_bounds__(512, kSymOccupancyWide) void lm_sym_pair_wide_kernel(SymArgs<T> a)
{
    int64_t X, Y;
    sym_superblocks(blockIdx.x, a.nsb, X, Y);
    sym_superblock_pair<T, DIM, KER, true, false, kSymRowsWide>(a.q, a.p, a.n, a.n, a.nsb, X, Y, a.kq, a.wscale,
                                                               a.part, nullptr, 0.0, nullptr, blockIdx.x);
}

// Batched: workgroup b takes item sym_items[b] = (problem, X, Y, S) of the concatenated
// (dim, ntot) arrays; the problem's partial sums start at part + part_off[problem].
template <class T, int DIM, int KER, bool FORCE>
__global__ __launch_bounds__(512, kSymOccupancy) void lm_batch_sym_kernel(BatchArgs<T> a)
{
    const int4 w = a.sym_items[blockIdx.x];
    const int64_t off = a.offs[w.x];
    const int64_t nb = a.offs[w.x + 1] - off;
    sym_superblock_pair<T, DIM, KER, FORCE, false, kSymRows>(a.q + off, a.p + off, a.ntot, nb, w.w, w.y, w.z, a.kq,
                                                             a.wscale, a.part + a.part_off[w.x], nullptr, 0.0, nullptr,
                                                             0);
}

template <class T, int DIM, int KER, bool FORCE>
hipError_t launch_sym_t(const SymArgs<T>& a, int waves, hipStream_t st)
{
    constexpr int EC = FORCE ? 2 * DIM : DIM;
    const int64_t S = a.nsb;
    const dim3 grid((unsigned)(S * (S + 1) / 2));
    if (a.rows == kSymRowsWide) {
        if constexpr (FORCE) {
            if (a.box == nullptr) {
                const size_t lds = sym_lds_bytes<T, DIM>(waves, EC);
                hipLaunchKernelGGL((lm_sym_pair_wide_kernel<T, DIM, KER>), grid, dim3(64 * waves), lds, st, a);
                return hipGetLastError();
            }
        }
        // the same superblocks with two row tiles per wave and twice the waves (velocity-only
        // sums, e.g. the K x of a CG solve, run the two-row kernel)
        waves = waves * kSymRowsWide / kSymRows;
    } else if (a.rows != kSymRows) {
        return hipErrorInvalidValue;
    }
    const size_t lds = sym_lds_bytes<T, DIM>(waves, EC);
    const dim3 block(64 * waves);
    if (a.box == nullptr) {
        hipLaunchKernelGGL((lm_sym_pair_kernel<T, DIM, KER, FORCE, false>), grid, block, lds, st, a);
    } else if constexpr (FORCE) {
        // tile skipping: sums with forces (the shoot's stages)
        hipLaunchKernelGGL((lm_sym_pair_kernel<T, DIM, KER, FORCE, true>), grid, block, lds, st, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

template <class T>
hipError_t launch_sym_pair(int dim, int kernel, bool force, const SymArgs<T>& a, int waves, hipStream_t st)
{
    if (dim == 2) {
        if (kernel == LM_KERNEL_CONON)
            return force ? launch_sym_t<T, 2, LM_KERNEL_CONON, true>(a, waves, st)
                         : launch_sym_t<T, 2, LM_KERNEL_CONON, false>(a, waves, st);
        return force ? launch_sym_t<T, 2, LM_KERNEL_GAUSS, true>(a, waves, st)
                     : launch_sym_t<T, 2, LM_KERNEL_GAUSS, false>(a, waves, st);
    }
    if (kernel == LM_KERNEL_CONON)
        return force ? launch_sym_t<T, 3, LM_KERNEL_CONON, true>(a, waves, st)
                     : launch_sym_t<T, 3, LM_KERNEL_CONON, false>(a, waves, st);
    return force ? launch_sym_t<T, 3, LM_KERNEL_GAUSS, true>(a, waves, st)
                 : launch_sym_t<T, 3, LM_KERNEL_GAUSS, false>(a, waves, st);
}

template hipError_t launch_sym_pair<double>(int, int, bool, const SymArgs<double>&, int, hipStream_t);

template <class T, int DIM, int KER, bool FORCE>
static hipError_t launch_batch_sym_t(const BatchArgs<T>& a, hipStream_t st)
{
    constexpr int EC = FORCE ? 2 * DIM : DIM;
    const int waves = a.sym_waves;
    const size_t lds = sym_lds_bytes<T, DIM>(waves, EC);
    hipLaunchKernelGGL((lm_batch_sym_kernel<T, DIM, KER, FORCE>), dim3((unsigned)a.nsym), dim3(64 * waves), lds, st, a);
    return hipGetLastError();
}

template <class T>
hipError_t launch_batch_sym(int dim, int kernel, bool force, const BatchArgs<T>& a, hipStream_t st)
{
    if (a.nsym == 0) return hipSuccess;
    if (dim == 2) {
        if (kernel == LM_KERNEL_CONON)
            return force ? launch_batch_sym_t<T, 2, LM_KERNEL_CONON, true>(a, st)
                         : launch_batch_sym_t<T, 2, LM_KERNEL_CONON, false>(a, st);
        return force ? launch_batch_sym_t<T, 2, LM_KERNEL_GAUSS, true>(a, st)
                     : launch_batch_sym_t<T, 2, LM_KERNEL_GAUSS, false>(a, st);
    }
    if (kernel == LM_KERNEL_CONON)
        return force ? launch_batch_sym_t<T, 3, LM_KERNEL_CONON, true>(a, st)
                     : launch_batch_sym_t<T, 3, LM_KERNEL_CONON, false>(a, st);
    return force ? launch_batch_sym_t<T, 3, LM_KERNEL_GAUSS, true>(a, st)
                 : launch_batch_sym_t<T, 3, LM_KERNEL_GAUSS, false>(a, st);
}

template hipError_t launch_batch_sym<double>(int, int, bool, const BatchArgs<double>&, hipStream_t);
template hipError_t launch_batch_sym<float>(int, int, bool, const BatchArgs<float>&, hipStream_t);
template hipError_t launch_sym_pair<float>(int, int, bool, const SymArgs<float>&, int, hipStream_t);

}  // namespace lm
