// lm_internal.h -- declarations shared by the kernels (lm_kernels.hip) and the host API
// (lm_api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/liblm.h"

namespace lm {

// Launch shape (measured on MI355X at N = 65536, 3-D, FP64): four waves per workgroup, four
// sources per unrolled loop body, and at least 16384 workgroups, so that each wave streams a
// chunk of about a thousand sources.  Short chunks stay in the scalar cache while the four
// waves of a CU's workgroups reuse them; one chunk per wave of the whole source range (the
// 1024-workgroup shape) ran 9-12% slower.
#ifndef LM_WAVES
#define LM_WAVES 4
#endif
#ifndef LM_UNROLL
#define LM_UNROLL 4
#endif
#ifndef LM_MIN_GROUPS
#define LM_MIN_GROUPS 16384
#endif

constexpr int kTile = 64;          // targets per workgroup (one per lane)
constexpr int kWaves = LM_WAVES;   // wavefronts per workgroup
constexpr int kUnroll = LM_UNROLL; // sources per unrolled loop body

enum EpiKind : int {
    EPI_STORE = 0,   // out_q = v + tau p_i, out_p = f            (right-hand side, K x)
    EPI_RK1 = 1,     // RK4 stage 1: acc = k1,    out = base + dt/2 k1
    EPI_RK2 = 2,     // RK4 stage 2: acc += 2k2,  out = base + dt/2 k2
    EPI_RK3 = 3,     // RK4 stage 3: acc += 2k3,  out = base + dt k3
    EPI_RK4 = 4      // RK4 stage 4: out = base + dt/6 (acc + k4)
};

template <class T>
struct EpiArgs {
    int kind;
    double dt;
    double tau;
    const T* in_p;     // target momenta (tau term), (dim, nt)
    const T* base_q;   // state at the start of the step
    const T* base_p;
    T* acc_q;          // RK4 running sum k1 + 2k2 + 2k3
    T* acc_p;
    T* out_q;          // stage output
    T* out_p;
    // qscale > 0 (a shoot on positions in the exponent's units): RK1-RK3 write their stage
    // output positions times qscale (the next stage's pair-sum input), and RK4, which writes
    // the state itself, also writes it times qscale to out_qs (the next step's first input)
    double qscale;
    T* out_qs;
};

template <class T>
struct PairArgs {
    const T* qs;       // sources (dim, ns)
    const T* ps;
    const T* qt;       // targets (dim, nt)
    const T* pt;
    int64_t nt, ns;
    int64_t jchunk;    // sources per wave chunk
    double kq;         // base-2 exponent scale: conon -log2(e)/sigma, Gaussian -log2(e)/sigma^2
    double wscale;     // force-weight constant: conon 1/sigma, Gaussian 2/sigma^2
    // tscale > 0: the sources are in the exponent's units (q' = k q, k = -kq for the conon,
    // sqrt(-kq) for the Gaussian) and the targets are multiplied by tscale as they are loaded
    // (1 when they are in those units already); wscale then carries the Gaussian's 1/k.  Only
    // the one-sided kernel without tile skipping takes this form.
    double tscale;
    T* part;           // split partial sums (nsplit, 2 dim, nt), used when nsplit > 1, in T (each
                       // partial is a double sum rounded once; they are added in double)
    const double* box_s;   // cutoff mode: source tile boxes (8 doubles per 64-point tile), else null
    const double* box_t;   // cutoff mode: target tile boxes
    double rc2;            // cutoff radius squared
    EpiArgs<T> epi;
};

// Reverse mode (lm_adjoint.hip).
enum AdjKind : int {
    ADJ_STORE = 0,   // lam = Ybar (a plain vector-Jacobian product)
    ADJ_FIRST = 1,   // RK4 stage 4: lam = abar + Ybar, nxt = ca abar + cy Ybar
    ADJ_MID = 2,     // stages 3 and 2: lam += Ybar, nxt = ca abar + cy Ybar
    ADJ_LAST = 3     // stage 1: lam += Ybar
};

struct AdjEpi {
    int kind;
    double cscale;          // Ybar = cscale * J^T (cot_q, cot_p)
    double ca, cy;
    double tau;
    const double* cot_q;    // the cotangent the VJP is taken of (its q part feeds the tau term)
    const double* abar_q;   // cotangent of the RK4 step output
    const double* abar_p;
    double* lam_q;          // cotangent of the step input (running sum)
    double* lam_p;
    double* nxt_q;          // cotangent of the next (earlier) stage
    double* nxt_p;
};

struct VjpArgs {
    const double* q;        // stage input (dim, n)
    const double* p;
    double* pack;           // 4 dim n doubles: the sources (q_j, p_j, a_j, b_j) interleaved
    const double* a;        // cotangent of dq/dt (dim, n)
    const double* b;        // cotangent of dp/dt
    int64_t n;
    int64_t jchunk;
    double kq;              // base-2 exponent scale (conon -log2(e)/sigma, Gaussian -log2(e)/sigma^2)
    double c1, c2;          // conon: c1 = 1/sigma; Gaussian: c1 = 2/sigma^2, c2 = -4/sigma^4
    double* part;
    AdjEpi epi;
};

// Batched pair sums (problems concatenated in one (dim, ntot) array; see lm_batch_pair_kernel).
template <class T>
struct BatchArgs {
    const T* q;              // stage input (dim, ntot)
    const T* p;
    int64_t ntot;
    const int64_t* offs;     // problem b owns [offs[b], offs[b+1])
    const int4* items;       // (problem, first target, chunk, chunks), sorted by cost
    int32_t nitems;
    const int64_t* part_off; // split problems: offset of their partials in part (elements)
    T* part;                 // partial sums in T, added in double
    double kq;
    double wscale;
    EpiArgs<T> epi;          // over the concatenated arrays (n = ntot)
    const int4* sym_items;   // symmetric problems: (problem, X, Y, S) superblock pairs, one per
    int32_t nsym;            //   workgroup of sym_waves waves (lm_batch_sym_kernel)
    int sym_waves;
};

template <class T>
hipError_t launch_batch_pair(int dim, int kernel, bool force, const BatchArgs<T>& a, const int4* fin, int32_t nfin,
                             int groups, hipStream_t st);
// The symmetric items of a batch (lm_sym.hip); their partial sums are added by the batch's
// finish launch.
template <class T>
hipError_t launch_batch_sym(int dim, int kernel, bool force, const BatchArgs<T>& a, hipStream_t st);
template <class TX>
hipError_t launch_batch_maxabsdiff(const TX* x, const double* y, int dim, int64_t ntot, const int64_t* offs, int nprob,
                                   double* out, hipStream_t st);
hipError_t launch_batch_dot(const double* x, const double* y, int dim, int64_t ntot, const int64_t* offs, int nprob,
                            double* out, hipStream_t st);
hipError_t launch_batch_axpy(double* p, const double* x, double h, int dim, int64_t ntot, const int64_t* offs,
                             const int* active, int nprob, hipStream_t st);
hipError_t launch_batch_copy_f32_to_f64(double* dst, const float* src, int dim, int64_t ntot, const int64_t* offs,
                                        const int* flag, int nprob, hipStream_t st);

// Whole shoots of problems of at most kSmallMax points, one workgroup each (see
// lm_small_shoot_kernel): (q, p) advanced in place by `steps` RK4 steps of size dt.
constexpr int kSmallMax = 256;
// Whether a shoot of n points takes that one-workgroup path (without tile skipping): up to 128
// points.  The environment variable LM_SMALL = 0 or 1 overrides the size rule (1: every size up
// to kSmallMax), for tuning and tests.  Defined in lm_kernels.hip.
bool small_path(int64_t n, int dim, bool fp32);

template <class T>
struct SmallShootArgs {
    T* q;                    // (dim, ntot), in place
    T* p;
    int64_t ntot;
    const int64_t* offs;     // problem b owns [offs[b], offs[b+1]); null: one problem of ntot
    double dt;
    int steps;
    double kq;
    double wscale;
    double tau;
};

template <class T>
hipError_t launch_small_shoot(int dim, int kernel, const SmallShootArgs<T>& a, int problems, hipStream_t st);

struct PairPlan {
    int64_t itiles;
    int nsplit;          // partial-sum slots per target (1: none)
    int64_t jchunk;
    int sym_waves;       // > 0: symmetric kernel (lm_sym.hip) with this many waves per workgroup
    int sym_rows;        // and this many row tiles per wave
    int64_t sym_nsb;     // its superblock count S (nsplit = S + 1)
};

// sym_ok: the targets are the sources (one point set, every pair, double precision), so the
// symmetric kernel may be chosen.  The environment variable LM_SYM overrides the size rule:
// "0" never, "1" always (for tests of small sizes).
// What a symmetric launch computes (its size rule differs): double- or single-precision sums,
// or their vector-Jacobian product (double).
enum SymKind : int { SYM_F64 = 0, SYM_F32 = 1, SYM_VJP = 2 };

PairPlan plan_pair(int64_t nt, int64_t ns, bool cut, bool sym_ok = false, int kind = SYM_F64);

// Symmetric pair sums of one point set (lm_sym.hip).
template <class T>
struct SymArgs {
    const T* q;          // (dim, n)
    const T* p;
    int64_t n;
    int64_t nsb;         // superblocks of rows * waves tiles
    int rows;            // row tiles per wave: kSymRows, or kSymRowsWide (double, forces, no cutoff)
    double kq;
    double wscale;
    T* part;             // (nsb + 1, 2 dim, n) partial sums in T, added in double
    const double* box;   // tile skipping: tile boxes (8 doubles per 64-point tile), else null
    double rc2;          // cutoff radius squared
    uint8_t* flags;      // tile skipping: one byte per superblock pair, 0 = nothing written
};

// Bytes of the superblock-pair flags that follow the partial sums of a symmetric launch with
// tile skipping, in doubles.
inline int64_t sym_flag_elems(int64_t nsb) { return (nsb * (nsb + 1) / 2 + 7) / 8; }

struct SymPlan {
    int waves = 0;       // 0: not worth it (too few wavefronts) or too large
    int rows = 2;        // row tiles per wave
    int64_t nsb = 0;
};

// Size rule (measured on MI355X, 3-D conon, FP64, one stage): from 128 tiles (N = 8192) one
// wave per workgroup, from 192 tiles (N = 12288) two, from 768 tiles (N = 49152) four; below,
// the one-sided kernel.
// At N = 16384 the symmetric kernel with two waves takes 298 us against 361, at 32768 997
// against 1371, at 65536 (four waves) 3760 against 5425.
constexpr int kSymMaxWaves = 8;
#ifndef LM_SYM_ROWS
#define LM_SYM_ROWS 2
#endif
constexpr int kSymRows = LM_SYM_ROWS;   // 64-point row tiles per wavefront
#ifndef LM_SYM_OCC
#define LM_SYM_OCC (LM_SYM_ROWS > 2 ? 3 : 4)
#endif
constexpr int kSymOccupancy = LM_SYM_OCC;   // wavefronts per SIMD the register budget allows
constexpr int kSymRowsWide = 4;             // the widest tier (lm_sym_pair_wide_kernel)
constexpr int kSymOccupancyWide = 3;
#ifndef LM_SYM_MIN_TILES
#define LM_SYM_MIN_TILES 192
#endif
constexpr int64_t kSymMinTiles = LM_SYM_MIN_TILES;
constexpr int64_t kSymWideTiles = 768;
// one wave per workgroup from 128 tiles (N = 8192: 3-D conon 92 against 101 us, 3-D Gaussian 79
// against 80, 2-D conon 78 against 86)
constexpr int64_t kSymOneWaveTiles = 128;
// With tile skipping (3-D Gaussian, cutoff where the kernel is 1e-16): at N = 65536 the
// symmetric kernel takes 502 us per stage against 574 one-sided (conon: 3784 against 5542),
// at N = 16384 149 against 120.
constexpr int64_t kSymCutTiles = 768;
// Single precision (column sums in registers, two row tiles per wave, float partial sums),
// 3-D conon sphere shoots, us per stage, one-sided against symmetric with one | two | four
// waves: N = 12288 81.6 against 89.9 | 97.2 | 121.1, 16384 137.6 against 133.0 | 139.2 |
// 164.4, 20480 199.8 against 189.2 | 192.3 | 213.4, 24576 280.8 against 258.2 | 261.2 | 261.9,
// 32768 501.7 against 435.6 | 421.7 | 439.4; with double partial sums 49152 1073 against
// 956 (two) | 911-914 (four), 65536 1945 against 1708 | 1603, 98304 4215-4220 against
// 3769-3779 | 3516.  Four rows per wave: 1686-1695 at 65536 (two waves).
#ifndef LM_SYM_MIN_TILES_F32
#define LM_SYM_MIN_TILES_F32 256
#endif
constexpr int64_t kSymMinTilesF32 = LM_SYM_MIN_TILES_F32;
constexpr int64_t kSymF32TwoWaveTiles = 512;
constexpr int64_t kSymF32FourWaveTiles = 768;
// The VJP (heavier pairs, 154-162 VGPRs) gains from 128 tiles on: at N = 8192 one wave per
// workgroup 136 us against 158 one-sided, at 16384 two waves 415 against 545, at 65536 two
// waves 6436 against 9632 (four: 6594).
constexpr int64_t kSymVjpMinTiles = 128;
constexpr int64_t kSymVjpTwoWaveTiles = 192;
constexpr int64_t kSymMaxPartBytes = (int64_t)16 << 30;

// cut: tile skipping (the wide tier has no tile skipping)
SymPlan plan_sym(int64_t n, bool force, int kind, bool cut = false);
template <class T>
hipError_t launch_sym_pair(int dim, int kernel, bool force, const SymArgs<T>& a, int waves, hipStream_t st);

template <class T>
hipError_t launch_pair(int dim, int kernel, bool force, const PairArgs<T>& a, const PairPlan& pl,
                       hipStream_t st);

int reduce_blocks(int64_t m);

hipError_t launch_vjp(int dim, int kernel, const VjpArgs& a, const PairPlan& pl, hipStream_t st);
// The symmetric form (lm_sym_vjp.hip): partial sums in (nsb + 1) slots of a.part, without the
// epilogue (launch_vjp adds them).
hipError_t launch_sym_vjp(int dim, int kernel, const VjpArgs& a, int waves, int64_t nsb, hipStream_t st);
hipError_t launch_scale(double* y, double alpha, const double* x, int64_t m, hipStream_t st);
// y = (T)(alpha * x), m elements
template <class T>
hipError_t launch_scaled_copy(T* y, const T* x, double alpha, int64_t m, hipStream_t st);

template <class TA, class TB>
hipError_t launch_maxabsdiff(const TA* x, const TB* y, int64_t m, double* partial, double* out, hipStream_t st);

hipError_t launch_dots(const double* x, const double* y, int64_t n, int ncomp, double* partial, double* out,
                       hipStream_t st);
hipError_t launch_cg_update_xr(double* x, double* r, const double* p, const double* ap, const double* rr,
                               const double* pap, int64_t n, int ncomp, hipStream_t st);
hipError_t launch_cg_update_p(double* p, const double* r, const double* rr_new, const double* rr, int64_t n,
                              int ncomp, hipStream_t st);
hipError_t launch_axpy(double* y, const double* x, double alpha, const double* z, int64_t m, hipStream_t st);
hipError_t launch_zero(double* y, int64_t m, hipStream_t st);
hipError_t launch_sub(double* y, const double* x, const double* z, int64_t m, hipStream_t st);

template <class TO, class TI>
hipError_t launch_convert(TO* y, const TI* x, int64_t m, hipStream_t st);

// Dense K(X) = L L^T (lower triangle of a row-major n x n buffer) with the inverses of the
// 128 x 128 diagonal blocks (dense_linv_elems doubles); *info != 0 flags a non-positive pivot.
// n must stay below kDenseMaxN: the trailing update addresses 128 rows of the matrix with
// 31-bit byte offsets (a factor that size would need 35 TB anyway).
constexpr int64_t kDenseMaxN = (int64_t)1 << 21;
int dense_panels(int64_t n);
int64_t dense_linv_elems(int64_t n);
// f32_update: the trailing updates of 1024 rows or more multiply in single precision (a factor
// for solves that only steer an iteration; about cond(K) times 1e-6 relative).  panel
// (nullable, dense_panel_f32_elems(n) floats): a buffer for the float copy of each update's
// operand columns, which the update then stages at half the bytes (the same result).
int64_t dense_panel_f32_elems(int64_t n);
hipError_t launch_dense_factor(int dim, int kernel, double kq, double tau, const double* X, int64_t n, double* K,
                               double* Linv, int* info, hipStream_t st, bool f32_update = false,
                               float* panel = nullptr);
// y <- (L L^T)^{-1} y for dim component vectors (component c at y + c * ldy), in place.
hipError_t launch_dense_solve(const double* L, const double* Linv, int64_t n, int dim, double* y, int64_t ldy,
                              hipStream_t st);
// Superblock sweeps (three launches per 8 diagonal blocks instead of one per block): the
// inverses of the factor's diagonal superblocks (dense_super_elems doubles, built by
// launch_dense_super once the factor is done), then y <- (L L^T)^{-1} y as above with
// dense_solve_scratch_elems doubles of scratch.  dense_super_default: whether n has more
// than one superblock.
int64_t dense_super_elems(int64_t n);
int64_t dense_solve_scratch_elems(int64_t n);
bool dense_super_default(int64_t n);
hipError_t launch_dense_super(const double* L, const double* Linv, int64_t n, double* W, hipStream_t st);
hipError_t launch_dense_solve_super(const double* L, const double* Linv, const double* W, int64_t n, int dim,
                                    double* y, int64_t ldy, double* scratch, hipStream_t st);

// Batched solves, one workgroup per flagged problem (every flagged problem must have at most
// batch_solve_max() points): y_b <- (L_b L_b^T)^{-1} y_b in the batch's (dim, ntot) layout.
int batch_solve_max();
hipError_t launch_batch_dense_solve(const double* L, const int64_t* loff, const double* Linv, const int64_t* ioff,
                                    const int64_t* offs, int nprob, int dim, int64_t ntot, double* y, const int* flag,
                                    hipStream_t st);

// Batched wide sweeps: the per-block sweeps for many problems of a batch at once (launch k
// serves block k of every listed problem, many workgroups per problem).  The item lists of
// every launch are built on the host once per set of problems (batch_wide_plan) and uploaded
// by the caller; flag[b] = 0 skips problem b.
struct BatchWidePlan {
    std::vector<int4> items;
    std::vector<int> fwd, bwd;   // start of each launch's list, maxnb + 1 entries each
    int maxnb = 0;
};
void batch_wide_plan(const int64_t* offs, const std::vector<int>& probs, BatchWidePlan* pl);
hipError_t launch_batch_wide_solve(const double* L, const int64_t* loff, const double* Linv, const int64_t* ioff,
                                   const int64_t* offs, int dim, int64_t ntot, double* y, const int* flag,
                                   const int4* items, const BatchWidePlan& pl, hipStream_t st);

// Matches with single-precision shoots: a shoot whose residual is not below kF32Stall times
// the previous one has reached the floor of single-precision shoots (the feedback iteration
// otherwise shrinks the residual by a factor of about 2 to 4 per update), so the same momenta
// are re-shot in double precision and the match stays there.  On the 65536-point sphere the
// floor is about 3e-6 and the residual ratios before it 0.24 to 0.61.
constexpr double kF32Stall = 0.9;

int64_t tiles_of(int64_t n);     // 64-point tiles covering n points
int64_t sort_pad(int64_t n);     // power of two >= max(n, 2)

// Bounding boxes of the 64-point tiles of q (8 doubles per tile: lo[4], hi[4]).
template <class T>
hipError_t launch_tile_boxes(int dim, const T* q, int64_t n, double* box, hipStream_t st);

// perm = the order of the points sorted by the Morton code of their position in the global
// bounding box.  box: tiles_of(n)*8 doubles; gbox: 8 doubles; keys: sort_pad(n) words.
template <class T>
hipError_t launch_morton_order(int dim, const T* q, int64_t n, double* box, double* gbox, uint64_t* keys,
                               int64_t* perm, hipStream_t st);

// out[c][i] = in[c][perm[i]] (gather) or out[c][perm[i]] = in[c][i] (scatter)
template <class TO, class TI>
hipError_t launch_permute(TO* out, const TI* in, const int64_t* perm, int64_t n, int dim, bool scatter, hipStream_t st);

}  // namespace lm
