// lm_batch.hip -- host side of the batched entry points (many independent problems of
// uneven size in one call; see include/liblm.h).
//
// A batch is planned once per call: every problem's 64-target tiles, times the source
// chunks of its size bucket, become work items (problem, first target, chunk, chunks),
// sorted by cost (the chunk length) from largest to smallest.  Each RK4 stage of the whole
// batch is then one launch of lm_batch_pair_kernel over that list (plus lm_batch_finish_kernel
// when some bucket splits its sources).  The stage sequence of a shoot can be captured once
// into a hipGraph and replayed, which removes the per-launch host cost that dominates small
// problems.  The autotuner picks the grid size, the per-bucket source splits and the steps
// per graph by timing them on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "lm_host.h"
#include "lm_internal.h"

namespace {

// Default size from which a batch's problems use the symmetric kernel (the autotuner's choice
// on the 256-curve workload in both precisions: 256; FP64 with two waves per workgroup, FP32
// with one or two).
constexpr int32_t kDefaultSymMin = 256;

using namespace lmh;

lm_status check_offs(int32_t B, const int64_t* offs, int64_t* ntot, int64_t* nmax)
{
    if (B < 1) return fail(LM_EINVAL, "B must be >= 1 (got %d)", B);
    if (!offs) return fail(LM_EINVAL, "offs is NULL");
    if (offs[0] != 0) return fail(LM_EINVAL, "offs[0] must be 0");
    int64_t mx = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t nb = offs[b + 1] - offs[b];
        if (nb < 1) return fail(LM_EINVAL, "problem %d is empty or offs is not increasing", b);
        if (nb > ((int64_t)1 << 30)) return fail(LM_EINVAL, "problem %d has more than 2^30 points", b);
        mx = std::max(mx, nb);
    }
    if (offs[B] > kMaxN) return fail(LM_EINVAL, "total size exceeds 2^34");
    *ntot = offs[B];
    *nmax = mx;
    return LM_OK;
}

lm_status check_tuning(const lm_batch_tuning* t, int64_t nmax)
{
    for (int k = 0; k < LM_BATCH_BUCKETS; ++k) {
        if (t->split[k] < 1 || t->split[k] > 64) return fail(LM_EINVAL, "tuning split[%d] must be in 1..64", k);
        if (t->bucket_max[k] < 1 || (k > 0 && t->bucket_max[k] < t->bucket_max[k - 1]))
            return fail(LM_EINVAL, "tuning bucket_max must be positive and ascending");
    }
    if (t->bucket_max[LM_BATCH_BUCKETS - 1] < nmax)
        return fail(LM_EINVAL, "tuning bucket_max[%d] = %lld is below the largest problem (%lld)",
                    LM_BATCH_BUCKETS - 1, (long long)t->bucket_max[LM_BATCH_BUCKETS - 1], (long long)nmax);
    if (t->groups < 0 || t->groups > (1 << 20)) return fail(LM_EINVAL, "tuning groups must be in 0..2^20");
    if (t->graph_steps < 0) return fail(LM_EINVAL, "tuning graph_steps must be >= 0");
    if (t->sym_min < 0) return fail(LM_EINVAL, "tuning sym_min must be >= 0");
    if (t->sym_waves != 1 && t->sym_waves != 2 && t->sym_waves != 4 && t->sym_waves != 8)
        return fail(LM_EINVAL, "tuning sym_waves must be 1, 2, 4 or 8");
    return LM_OK;
}

void default_tuning(lm_batch_tuning* t, int64_t nmax)
{
    std::memset(t, 0, sizeof *t);
    const int64_t bmax[LM_BATCH_BUCKETS] = {128, 512, 2048, 0};
    for (int k = 0; k < LM_BATCH_BUCKETS; ++k) {
        t->bucket_max[k] = bmax[k];
        t->split[k] = 1;
    }
    t->bucket_max[LM_BATCH_BUCKETS - 1] = std::max<int64_t>(nmax, 2049);
    t->groups = 0;
    t->graph_steps = 10;
    t->sym_min = kDefaultSymMin;
    t->sym_waves = 2;
    t->stage_us = 0.0;
}

// Compute units of the current device (256 on MI355X when the query fails).
int device_cus()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        return prop.multiProcessorCount;
    return 256;
}

// Fewest waves per launch of a batched match's shoots: kFillWavesPerSimd per SIMD (four SIMDs
// per CU); LM_BATCH_FILL overrides the per-SIMD figure (0 keeps the tuning's shape).  On the
// tail of the 256-curve match (the 1 to 16 largest curves, 3229 to 4065 points), per 100-step
// shoot: in single precision 10.5-48.3 ms against 53-59 ms with the whole batch's splits, within
// 12% of the best split a sweep found; in double precision, one-wave superblocks for the 1, 2
// and 4 largest took 19.4, 21.1 and 30.1 ms against 28.2, 40.4 and 42.5 ms with two waves.
constexpr int kFillWavesPerSimd = 2;

int64_t match_min_waves()
{
    int64_t per_simd = kFillWavesPerSimd;
    if (const char* e = std::getenv("LM_BATCH_FILL")) per_simd = std::max(0L, std::strtol(e, nullptr, 10));
    return per_simd * 4 * device_cus();
}

int bucket_of(const lm_batch_tuning& t, int64_t nb)
{
    for (int k = 0; k < LM_BATCH_BUCKETS; ++k)
        if (nb <= t.bucket_max[k]) return k;
    return LM_BATCH_BUCKETS - 1;
}

// Work list of a batch for one launch shape, on the device.
struct BatchPlan {
    int4* sym_items_d = nullptr;   // symmetric problems' superblock pairs, largest first
    int32_t nsym = 0;
    int sym_waves = 1;
    int32_t B = 0;
    int64_t ntot = 0;
    int dim = 0;
    int groups = 1;
    const int64_t* offs_d = nullptr;
    int4* items_d = nullptr;
    int32_t nitems = 0;
    int4* fin_d = nullptr;
    int32_t nfin = 0;
    int64_t* part_off_d = nullptr;
    double* part = nullptr;
};

// Builds the work list on the host and uploads it (the host vectors are copied before this
// returns: the copies are synchronous with respect to the host).
// include (nullable) selects the problems to plan.  min_waves > 0 asks for at least that many
// waves per launch: while the plan has fewer, the symmetric problems' workgroups are narrowed
// (half the waves, half the superblock side, down to one wave), then the one-sided problems'
// source splits are doubled together (each up to 64 chunks and at most one chunk per source
// point).  A tuning made for a whole batch can leave a few of its problems, the tail of a
// batched match, on a small part of the chip: one 4065-point problem split in two is 128 waves
// on 1024 SIMDs, and in double precision with two-wave superblocks 72.
lm_status make_plan(int dim, int32_t B, const int64_t* offs, const int64_t* offs_d, const lm_batch_tuning& t,
                    Workspace& ws, BatchPlan* pl, hipStream_t st, const std::vector<int>* include = nullptr,
                    int64_t min_waves = 0)
{
    struct Item {
        int4 w;
        int64_t cost;
    };
    std::vector<Item> items, sym;
    std::vector<int4> fin;
    std::vector<int64_t> part_off((size_t)B, -1);
    int64_t part_elems = 0;
    auto planned = [&](int32_t b) { return !include || (*include)[b]; };
    auto symmetric = [&](int64_t nb) { return t.sym_min > 0 && nb >= t.sym_min; };

    // waves of the symmetric problems with sw waves per workgroup (superblocks of kSymRows * sw
    // tiles, one workgroup per superblock pair)
    auto sym_waves_at = [&](int sw) {
        const int64_t sd = (int64_t)lm::kSymRows * sw;
        int64_t w = 0;
        for (int32_t b = 0; b < B; ++b) {
            const int64_t nb = offs[b + 1] - offs[b];
            if (!planned(b) || !symmetric(nb)) continue;
            const int64_t S = ((nb + 63) / 64 + sd - 1) / sd;
            w += S * (S + 1) / 2 * sw;
        }
        return w;
    };
    // source splits of the one-sided problems: the tuning's, times mult
    std::vector<int32_t> split((size_t)B, 0);
    for (int32_t b = 0; b < B; ++b) {
        const int64_t nb = offs[b + 1] - offs[b];
        if (planned(b) && !symmetric(nb)) split[b] = (int32_t)std::min<int64_t>(t.split[bucket_of(t, nb)], nb);
    }
    auto split_times = [&](int32_t b, int64_t mult) {
        return (int32_t)std::min<int64_t>({(int64_t)split[b] * mult, 64, offs[b + 1] - offs[b]});
    };
    auto one_sided_waves_at = [&](int64_t mult) {
        int64_t w = 0;
        for (int32_t b = 0; b < B; ++b)
            if (split[b] > 0) w += (offs[b + 1] - offs[b] + 63) / 64 * split_times(b, mult);
        return w;
    };
    int sw = t.sym_waves;
    int64_t mult = 1;
    if (min_waves > 0) {
        while (sw > 1 && sym_waves_at(sw) + one_sided_waves_at(1) < min_waves) sw /= 2;
        const int64_t symw = sym_waves_at(sw);
        while (symw + one_sided_waves_at(mult) < min_waves && one_sided_waves_at(2 * mult) > one_sided_waves_at(mult))
            mult *= 2;
    }
    const int64_t side = (int64_t)lm::kSymRows * sw;   // tiles per superblock

    for (int32_t b = 0; b < B; ++b) {
        if (include && !(*include)[b]) continue;
        const int64_t nb = offs[b + 1] - offs[b];
        if (symmetric(nb)) {
            // symmetric: one item per superblock pair (X <= Y), S + 1 partial-sum slots
            const int64_t nt = (nb + 63) / 64;
            const int64_t S = (nt + side - 1) / side;
            part_off[b] = part_elems;
            part_elems += (S + 1) * 2 * dim * nb;
            for (int64_t Y = 0; Y < S; ++Y)
                for (int64_t X = 0; X <= Y; ++X) {
                    const int64_t rows = std::min(side, nt - X * side), cols = std::min(side, nt - Y * side);
                    sym.push_back({make_int4(b, (int)X, (int)Y, (int)S), X == Y ? rows * (rows + 1) / 2 : rows * cols});
                }
            for (int64_t t0 = 0; t0 < nb; t0 += 64) fin.push_back(make_int4(b, (int)t0, (int)(S + 1), 0));
            continue;
        }
        const int32_t S = split_times(b, mult);
        const int64_t chunk = (nb + S - 1) / S;
        if (S > 1) {
            part_off[b] = part_elems;
            part_elems += (int64_t)S * 2 * dim * nb;
        }
        for (int64_t t0 = 0; t0 < nb; t0 += 64) {
            for (int32_t c = 0; c < S; ++c) {
                const int64_t len = std::max<int64_t>(0, std::min(chunk, nb - c * chunk));
                items.push_back({make_int4(b, (int)t0, c, S), len});
            }
            if (S > 1) fin.push_back(make_int4(b, (int)t0, S, 0));
        }
    }
    if (items.size() > (size_t)INT32_MAX) return fail(LM_EINVAL, "batch has too many work items");
    if (sym.size() > (size_t)INT32_MAX) return fail(LM_EINVAL, "batch has too many symmetric work items");
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::stable_sort(sym.begin(), sym.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<int4> w(items.size()), ws_sym(sym.size());
    for (size_t k = 0; k < items.size(); ++k) w[k] = items[k].w;
    for (size_t k = 0; k < sym.size(); ++k) ws_sym[k] = sym[k].w;
    pl->nsym = (int32_t)ws_sym.size();
    pl->sym_waves = sw;
    LM_TRY(ws.get(&pl->sym_items_d, std::max<int32_t>(pl->nsym, 1)));
    if (pl->nsym > 0)
        LM_HIP(hipMemcpyAsync(pl->sym_items_d, ws_sym.data(), ws_sym.size() * sizeof(int4), hipMemcpyHostToDevice, st));

    pl->B = B;
    pl->ntot = offs[B];
    pl->dim = dim;
    pl->offs_d = offs_d;
    pl->nitems = (int32_t)w.size();
    pl->nfin = (int32_t)fin.size();
    const int32_t natural = (pl->nitems + lm::kWaves - 1) / lm::kWaves;
    pl->groups = t.groups > 0 ? std::min(t.groups, natural) : natural;
    LM_TRY(ws.get(&pl->items_d, std::max<int32_t>(pl->nitems, 1)));
    LM_TRY(ws.get(&pl->fin_d, std::max<int32_t>(pl->nfin, 1)));
    LM_TRY(ws.get(&pl->part_off_d, B));
    LM_TRY(ws.get(&pl->part, std::max<int64_t>(part_elems, 1)));
    LM_HIP(hipMemcpyAsync(pl->items_d, w.data(), w.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    if (pl->nfin > 0)
        LM_HIP(hipMemcpyAsync(pl->fin_d, fin.data(), fin.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    LM_HIP(hipMemcpyAsync(pl->part_off_d, part_off.data(), part_off.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          st));
    // the host vectors die with this frame
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

lm_status upload_offs(int32_t B, const int64_t* offs, Workspace& ws, int64_t** offs_d, hipStream_t st)
{
    LM_TRY(ws.get(offs_d, B + 1));
    LM_HIP(hipMemcpyAsync(*offs_d, offs, (size_t)(B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

// One evaluation of the batched pair sums at (q, p) with epilogue e.
template <class T>
lm_status batch_eval(const lm_params* prm, const BatchPlan& pl, const T* q, const T* p, const lm::EpiArgs<T>& e,
                     hipStream_t st)
{
    lm::BatchArgs<T> a{};
    a.q = q;
    a.p = p;
    a.ntot = pl.ntot;
    a.offs = pl.offs_d;
    a.items = pl.items_d;
    a.nitems = pl.nitems;
    a.part_off = pl.part_off_d;
    a.part = reinterpret_cast<T*>(pl.part);   // sized in doubles; the partial sums are T
    a.sym_items = pl.sym_items_d;
    a.nsym = pl.nsym;
    a.sym_waves = pl.sym_waves;
    kernel_scales(prm, &a.kq, &a.wscale);
    a.epi = e;
    LM_HIP(lm::launch_batch_pair<T>(prm->dim, prm->kernel, true, a, pl.fin_d, pl.nfin, pl.groups, st));
    return LM_OK;
}

template <class T>
lm_status batch_rhs(const lm_params* prm, const BatchPlan& pl, const T* q, const T* p, T* dq, T* dp, hipStream_t st)
{
    lm::EpiArgs<T> e{};
    e.kind = lm::EPI_STORE;
    e.tau = prm->tau;
    e.in_p = p;
    e.out_q = dq;
    e.out_p = dp;
    return batch_eval<T>(prm, pl, q, p, e, st);
}

// RK4 stage buffers of a batch shoot.
template <class T>
struct ShootBufs {
    T *aq, *ap, *bq, *bp, *cq, *cp;
    lm_status alloc(Workspace& ws, int64_t m)
    {
        LM_TRY(ws.get(&aq, m));
        LM_TRY(ws.get(&ap, m));
        LM_TRY(ws.get(&bq, m));
        LM_TRY(ws.get(&bp, m));
        LM_TRY(ws.get(&cq, m));
        LM_TRY(ws.get(&cp, m));
        return LM_OK;
    }
};

// `count` RK4 steps of size dt of (q, p) in place (the same stage sequence as a single
// problem's shoot: y -> A -> B -> A -> y).
template <class T>
lm_status batch_steps(const lm_params* prm, const BatchPlan& pl, T* q, T* p, double dt, int32_t count,
                      const ShootBufs<T>& w, hipStream_t st)
{
    lm::EpiArgs<T> e{};
    e.dt = dt;
    e.tau = prm->tau;
    e.base_q = q;
    e.base_p = p;
    e.acc_q = w.cq;
    e.acc_p = w.cp;
    const T* in_q[4] = {q, w.aq, w.bq, w.aq};
    const T* in_p[4] = {p, w.ap, w.bp, w.ap};
    T* out_q[4] = {w.aq, w.bq, w.aq, q};
    T* out_p[4] = {w.ap, w.bp, w.ap, p};
    for (int32_t s = 0; s < count; ++s) {
        for (int k = 0; k < 4; ++k) {
            e.kind = lm::EPI_RK1 + k;
            e.in_p = in_p[k];
            e.out_q = out_q[k];
            e.out_p = out_p[k];
            LM_TRY(batch_eval<T>(prm, pl, in_q[k], in_p[k], e, st));
        }
    }
    return LM_OK;
}

// Side streams that start after the work already on a stream and that the stream then waits
// for (join).  Destroyed after st has drained.  Eight, although HIP gives a process four
// hardware queues by default and streams beyond four share them: measured on the 256-problem
// batch, the factors of all problems take 258-263 ms with eight streams and 329-350 ms with
// four.
constexpr int kFactorStreams = 8;

struct SideStreams {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> e;
    hipStream_t parent = nullptr;
    lm_status init(int n, hipStream_t st)
    {
        parent = st;
        hipEvent_t start;
        LM_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
        e.push_back(start);
        LM_HIP(hipEventRecord(start, st));
        for (int i = 0; i < n; ++i) {
            hipStream_t x;
            LM_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
            s.push_back(x);
            LM_HIP(hipStreamWaitEvent(x, start, 0));
        }
        return LM_OK;
    }
    lm_status join(hipStream_t st)
    {
        for (hipStream_t x : s) {
            hipEvent_t done;
            LM_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
            e.push_back(done);
            LM_HIP(hipEventRecord(done, x));
            LM_HIP(hipStreamWaitEvent(st, done, 0));
        }
        return LM_OK;
    }
    ~SideStreams()
    {
        for (hipStream_t x : s) (void)hipStreamSynchronize(x);
        for (hipStream_t x : s) (void)hipStreamDestroy(x);
        for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
};

// One side stream that forks from and joins a parent stream, as often as needed.
struct ForkJoin {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    lm_status init()
    {
        LM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        LM_HIP(hipEventCreateWithFlags(&a, hipEventDisableTiming));
        LM_HIP(hipEventCreateWithFlags(&b, hipEventDisableTiming));
        return LM_OK;
    }
    lm_status fork(hipStream_t st)
    {
        LM_HIP(hipEventRecord(a, st));
        LM_HIP(hipStreamWaitEvent(s, a, 0));
        return LM_OK;
    }
    lm_status join(hipStream_t st)
    {
        LM_HIP(hipEventRecord(b, s));
        LM_HIP(hipStreamWaitEvent(st, b, 0));
        return LM_OK;
    }
    ~ForkJoin()
    {
        if (s) (void)hipStreamSynchronize(s);
        if (s) (void)hipStreamDestroy(s);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Size above which a batched match solves a problem with the wide sweeps (many workgroups)
// rather than in lm_batch_solve_kernel (one workgroup); LM_BATCH_WIDE_MIN overrides it.
// Never above the one-workgroup kernel's limit.
constexpr int64_t kBatchWideMin = 1024;

int64_t batch_wide_min()
{
    int64_t v = kBatchWideMin;
    if (const char* e = std::getenv("LM_BATCH_WIDE_MIN")) v = std::max(0L, std::strtol(e, nullptr, 10));
    return std::min<int64_t>(v, lm::batch_solve_max());
}

// A captured sequence of RK4 steps, replayable on any stream.  The executable graph is
// destroyed only after the stream it was last launched on has drained, also when an error
// ends the call between two launches.
struct StepGraph {
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    bool launched = false;
    hipStream_t launch_stream = nullptr;
    hipError_t launch(hipStream_t st)
    {
        launched = true;
        launch_stream = st;
        return hipGraphLaunch(x, st);
    }
    void reset()
    {
        if (launched) (void)hipStreamSynchronize(launch_stream);
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        if (cs) (void)hipStreamDestroy(cs);
        x = nullptr;
        g = nullptr;
        cs = nullptr;
        launched = false;
    }
    ~StepGraph() { reset(); }
};

template <class T>
lm_status capture_steps(const lm_params* prm, const BatchPlan& pl, T* q, T* p, double dt, int32_t count,
                        const ShootBufs<T>& w, StepGraph* sg)
{
    sg->reset();
    LM_HIP(hipStreamCreateWithFlags(&sg->cs, hipStreamNonBlocking));
    LM_HIP(hipStreamBeginCapture(sg->cs, hipStreamCaptureModeThreadLocal));
    const lm_status s = batch_steps<T>(prm, pl, q, p, dt, count, w, sg->cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(sg->cs, &g);
    sg->g = g;
    LM_TRY(s);
    if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
    LM_HIP(hipGraphInstantiate(&sg->x, sg->g, nullptr, nullptr, 0));
    return LM_OK;
}

// Shoot of (q, p) in place over [0, t1].  With graph_steps > 0 the steps run as replays of
// a graph of graph_steps steps (plus directly launched remainder steps) and the call
// synchronizes.  cache (nullable) keeps the graph for later shoots of the same buffers,
// plan and step size; without it the graph is captured for this shoot alone.
template <class T>
lm_status batch_shoot_inplace(const lm_params* prm, const BatchPlan& pl, T* q, T* p, double t1, int32_t steps,
                              int32_t graph_steps, const ShootBufs<T>& w, hipStream_t st, StepGraph* cache = nullptr)
{
    const double dt = t1 / steps;
    if (graph_steps <= 0 || graph_steps > steps) return batch_steps<T>(prm, pl, q, p, dt, steps, w, st);
    StepGraph local;
    StepGraph* sg = cache ? cache : &local;
    if (!sg->x) LM_TRY(capture_steps<T>(prm, pl, q, p, dt, graph_steps, w, sg));
    const int32_t reps = steps / graph_steps;
    for (int32_t r = 0; r < reps; ++r) LM_HIP(sg->launch(st));
    LM_TRY(batch_steps<T>(prm, pl, q, p, dt, steps - reps * graph_steps, w, st));
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

template <class T>
lm_status shoot_batched_t(const lm_params* prm, int32_t B, const int64_t* offs, const T* q0, const T* p0, double t1,
                          int32_t steps, T* q1, T* p1, const lm_batch_tuning& tun, hipStream_t st)
{
    Workspace ws(st);
    int64_t* offs_d;
    LM_TRY(upload_offs(B, offs, ws, &offs_d, st));
    BatchPlan pl;
    LM_TRY(make_plan(prm->dim, B, offs, offs_d, tun, ws, &pl, st));
    const int64_t m = (int64_t)prm->dim * pl.ntot;
    if (q1 != q0) LM_HIP(hipMemcpyAsync(q1, q0, m * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (p1 != p0) LM_HIP(hipMemcpyAsync(p1, p0, m * sizeof(T), hipMemcpyDeviceToDevice, st));
    ShootBufs<T> w;
    LM_TRY(w.alloc(ws, m));
    return batch_shoot_inplace<T>(prm, pl, q1, p1, t1, steps, tun.graph_steps, w, st);
}

lm_status resolve_tuning(const lm_batch_tuning* t, int32_t B, const int64_t* offs, lm_batch_tuning* out,
                         int64_t* ntot)
{
    int64_t nmax;
    LM_TRY(check_offs(B, offs, ntot, &nmax));
    if (t) {
        LM_TRY(check_tuning(t, nmax));
        *out = *t;
    } else {
        default_tuning(out, nmax);
    }
    return LM_OK;
}

lm_status check_batch_params(const lm_params* prm)
{
    LM_TRY(check_params(prm));
    if (prm->cutoff != 0.0) return fail(LM_EUNSUPPORTED, "batched problems run all pairs (cutoff must be 0)");
    return LM_OK;
}

// ---------------------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------------------

// Median time (ms) of `reps` runs of fn() on the stream, after one untimed run.
template <class F>
lm_status time_ms(F fn, int reps, hipStream_t st, double* out)
{
    LM_TRY(fn());
    EventTimer tm;
    LM_TRY(tm.init());
    std::vector<double> t;
    for (int r = 0; r < reps; ++r) {
        LM_HIP(hipEventRecord(tm.ev[0], st));
        LM_TRY(fn());
        LM_HIP(hipEventRecord(tm.ev[1], st));
        LM_HIP(hipEventSynchronize(tm.ev[1]));
        t.push_back(tm.ms(0, 1));
    }
    std::sort(t.begin(), t.end());
    *out = t[t.size() / 2];
    return LM_OK;
}

template <class T>
lm_status autotune_t(const lm_params* prm, int32_t B, const int64_t* offs, const T* q, const T* p,
                     lm_batch_tuning* best, hipStream_t st)
{
    int64_t ntot, nmax;
    LM_TRY(check_offs(B, offs, &ntot, &nmax));
    default_tuning(best, nmax);
    Workspace ws(st);
    int64_t* offs_d;
    LM_TRY(upload_offs(B, offs, ws, &offs_d, st));
    const int64_t m = (int64_t)prm->dim * ntot;
    T *dq, *dp, *sq, *sp;
    LM_TRY(ws.get(&dq, m));
    LM_TRY(ws.get(&dp, m));
    LM_TRY(ws.get(&sq, m));
    LM_TRY(ws.get(&sp, m));
    ShootBufs<T> w;
    LM_TRY(w.alloc(ws, m));

    // one right-hand side of the batch with tuning t
    auto stage_time = [&](const lm_batch_tuning& t, double* ms) -> lm_status {
        Workspace pws(st);
        BatchPlan pl;
        LM_TRY(make_plan(prm->dim, B, offs, offs_d, t, pws, &pl, st));
        return time_ms([&]() { return batch_rhs<T>(prm, pl, q, p, dq, dp, st); }, 5, st, ms);
    };
    double cur;
    LM_TRY(stage_time(*best, &cur));

    // grid size: one wave per item, or a persistent grid of 1, 2, 4, 8 workgroups per CU
    const int cus = device_cus();
    for (int g : {1, 2, 4, 8}) {
        lm_batch_tuning t = *best;
        t.groups = g * cus;
        double ms;
        LM_TRY(stage_time(t, &ms));
        if (ms < cur) {
            cur = ms;
            *best = t;
        }
    }
    // the size from which problems go symmetric (0 = none), then its width
    {
        for (int sm : {0, 512, 1024, 2048, 4096}) {   // the default, 256, is the starting point
            lm_batch_tuning t = *best;
            t.sym_min = sm;
            double ms;
            LM_TRY(stage_time(t, &ms));
            if (ms < cur) {
                cur = ms;
                *best = t;
            }
        }
        if (best->sym_min > 0) {
            for (int sw : {1, 4}) {
                lm_batch_tuning t = *best;
                t.sym_waves = sw;
                double ms;
                LM_TRY(stage_time(t, &ms));
                if (ms < cur) {
                    cur = ms;
                    *best = t;
                }
            }
        }
    }
    // source splits of each occupied bucket, largest problems first
    std::vector<bool> used(LM_BATCH_BUCKETS, false);
    for (int32_t b = 0; b < B; ++b) used[bucket_of(*best, offs[b + 1] - offs[b])] = true;
    for (int k = LM_BATCH_BUCKETS - 1; k >= 0; --k) {
        if (!used[k]) continue;
        for (int s : {2, 4, 8}) {
            lm_batch_tuning t = *best;
            t.split[k] = s;
            double ms;
            LM_TRY(stage_time(t, &ms));
            if (ms < cur) {
                cur = ms;
                *best = t;
            }
        }
    }
    best->stage_us = cur * 1e3;

    // steps per graph, on a 20-step shoot of a copy of (q, p)
    {
        Workspace pws(st);
        BatchPlan pl;
        LM_TRY(make_plan(prm->dim, B, offs, offs_d, *best, pws, &pl, st));
        double bt = 0.0;
        int bg = 0;
        for (int gs : {0, 1, 5, 20}) {
            double ms;
            StepGraph sg;   // captured by the untimed first run, replayed by the timed ones
            LM_TRY(time_ms(
                [&]() -> lm_status {
                    LM_HIP(hipMemcpyAsync(sq, q, m * sizeof(T), hipMemcpyDeviceToDevice, st));
                    LM_HIP(hipMemcpyAsync(sp, p, m * sizeof(T), hipMemcpyDeviceToDevice, st));
                    return batch_shoot_inplace<T>(prm, pl, sq, sp, 1.0, 20, gs, w, st, &sg);
                },
                3, st, &ms));
            if (gs == 0 || ms < bt) {
                bt = ms;
                bg = gs;
            }
        }
        best->graph_steps = bg;
    }
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

// ---------------------------------------------------------------------------------------
// Batched Algorithm 1
// ---------------------------------------------------------------------------------------

lm_status match_batched(const lm_params* prm, const lm_match_opts* o, int32_t B, const int64_t* offs,
                        const double* X, const double* Y, double* p, double* q1_out, lm_match_info* info,
                        int32_t* status, const lm_batch_tuning& tun, hipStream_t st)
{
    const int dim = prm->dim;
    const bool f32 = prm->dtype == LM_F32;
    const bool may_switch = f32 && o->f32_switch > 0.0;
    Workspace ws(st);
    int64_t* offs_d;
    LM_TRY(upload_offs(B, offs, ws, &offs_d, st));
    const int64_t ntot = offs[B], m = (int64_t)dim * ntot;
    lm_params p64 = *prm, p32 = *prm;
    p64.dtype = LM_F64;
    p32.dtype = LM_F32;

    EventTimer tm;
    LM_TRY(tm.init());
    double shoot_ms = 0.0, solve_ms = 0.0, factor_ms = 0.0;

    // dense factors of every K(X_b) + tau I, each built from a contiguous copy of X_b
    std::vector<int64_t> loff((size_t)B), ioff((size_t)B);
    int64_t lsum = 0, isum = 0, nmax = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t nb = offs[b + 1] - offs[b];
        loff[b] = lsum;
        ioff[b] = isum;
        lsum += nb * nb;
        isum += lm::dense_linv_elems(nb);
        nmax = std::max(nmax, nb);
    }
    // the factors are independent: they are spread over kFactorStreams side streams (each
    // with its own copy buffer for X_b), which wait for the allocations on st and are waited
    // for by st
    const int ns = std::min<int32_t>(B, kFactorStreams);
    double *L, *Linv, *xb;
    int* finfo;
    int64_t *loff_d, *ioff_d;
    LM_TRY(ws.get(&L, lsum));
    LM_TRY(ws.get(&Linv, isum));
    LM_TRY(ws.get(&finfo, B));
    LM_TRY(ws.get(&xb, (int64_t)ns * dim * nmax));
    LM_TRY(ws.get(&loff_d, B));
    LM_TRY(ws.get(&ioff_d, B));
    LM_HIP(hipMemcpyAsync(loff_d, loff.data(), B * sizeof(int64_t), hipMemcpyHostToDevice, st));
    LM_HIP(hipMemcpyAsync(ioff_d, ioff.data(), B * sizeof(int64_t), hipMemcpyHostToDevice, st));
    double kq, wscale;
    kernel_scales(prm, &kq, &wscale);
    LM_HIP(hipEventRecord(tm.ev[0], st));
    {
        SideStreams side;
        LM_TRY(side.init(ns, st));
        for (int32_t b = 0; b < B; ++b) {
            const int64_t nb = offs[b + 1] - offs[b];
            hipStream_t fs = side.s[b % ns];
            double* x = xb + (int64_t)(b % ns) * dim * nmax;
            for (int c = 0; c < dim; ++c)
                LM_HIP(hipMemcpyAsync(x + c * nb, X + c * ntot + offs[b], nb * sizeof(double),
                                      hipMemcpyDeviceToDevice, fs));
            LM_HIP(lm::launch_dense_factor(dim, prm->kernel, kq, prm->tau, x, nb, L + loff[b], Linv + ioff[b],
                                           finfo + b, fs));
        }
        LM_TRY(side.join(st));
    }
    LM_HIP(hipEventRecord(tm.ev[1], st));
    std::vector<int> fi((size_t)B);
    LM_HIP(hipMemcpyAsync(fi.data(), finfo, B * sizeof(int), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));   // also retires the uploads of loff and ioff
    factor_ms = tm.ms(0, 1);

    // per-problem state: stat -1 while running; upd = momentum updates made; prec = 1 once
    // the problem's shoots are double precision
    std::vector<int32_t> stat((size_t)B, -1), upd((size_t)B, 0), prec((size_t)B, f32 ? 0 : 1);
    std::vector<double> res((size_t)B, 0.0), prevr((size_t)B, INFINITY);
    for (int32_t b = 0; b < B; ++b)
        if (fi[b] != 0) stat[b] = LM_ESINGULAR;

    double *qd, *pd, *e, *resid_d;
    int *flags_d;   // 4 x B: problems updated, one-workgroup solves, single-precision results, wide solves
    LM_TRY(ws.get(&qd, m));
    LM_TRY(ws.get(&pd, m));
    LM_TRY(ws.get(&e, m));
    LM_TRY(ws.get(&resid_d, B));
    LM_TRY(ws.get(&flags_d, 4 * (int64_t)B));
    float *xf = nullptr, *qf = nullptr, *pf = nullptr;
    ShootBufs<double> wd{};
    ShootBufs<float> wf{};
    LM_TRY(wd.alloc(ws, m));
    if (f32) {
        LM_TRY(ws.get(&xf, m));
        LM_TRY(ws.get(&qf, m));
        LM_TRY(ws.get(&pf, m));
        LM_TRY(wf.alloc(ws, m));
        LM_HIP((lm::launch_convert<float, double>(xf, X, m, st)));
    }
    std::vector<int> flags((size_t)4 * B, 0);
    int* upd_f = flags.data();
    int* solve_f = flags.data() + B;
    int* f32_f = flags.data() + 2 * B;
    int* wide_f = flags.data() + 3 * B;

    // work lists of the problems shot in each precision, rebuilt when those sets change
    std::vector<int> in64((size_t)B, -1), in32((size_t)B, -1);
    const int64_t fill = match_min_waves();
    std::unique_ptr<Workspace> pws64, pws32;
    BatchPlan pl64, pl32;
    StepGraph g64, g32;
    // problems above wide_min points are solved by the batched wide sweeps (many workgroups
    // per problem), on the match's stream, while lm_batch_solve_kernel takes the rest on a
    // side stream
    const int64_t wide_min = batch_wide_min();
    std::vector<int> wide_probs;
    for (int32_t b = 0; b < B; ++b)
        if (offs[b + 1] - offs[b] > wide_min && fi[b] == 0) wide_probs.push_back(b);
    lm::BatchWidePlan wplan;
    int4* witems = nullptr;
    ForkJoin fj;
    if (!wide_probs.empty()) {
        lm::batch_wide_plan(offs, wide_probs, &wplan);
        LM_TRY(ws.get(&witems, (int64_t)wplan.items.size()));
        LM_HIP(hipMemcpyAsync(witems, wplan.items.data(), wplan.items.size() * sizeof(int4), hipMemcpyHostToDevice,
                              st));
        LM_HIP(hipStreamSynchronize(st));   // the host list dies with this call's frame
        LM_TRY(fj.init());
    }

    // problems starting from zero momenta (the paper's starting guess) do not move: their
    // first shoot is the identity map, q(1) = X, and is not integrated
    std::vector<int> still((size_t)B, 0), nshoot((size_t)B, 0);
    {
        std::vector<double> pm((size_t)B, 1.0);
        LM_HIP(lm::launch_zero(e, m, st));
        LM_HIP(lm::launch_batch_maxabsdiff<double>(p, e, dim, ntot, offs_d, B, resid_d, st));
        LM_HIP(hipMemcpyAsync(pm.data(), resid_d, B * sizeof(double), hipMemcpyDeviceToHost, st));
        LM_HIP(hipStreamSynchronize(st));
        for (int32_t b = 0; b < B; ++b) still[b] = pm[b] == 0.0;
    }
    bool first = true;

    for (;;) {
        std::vector<int> want64((size_t)B), want32((size_t)B);
        bool any64 = false, any32 = false;
        for (int32_t b = 0; b < B; ++b) {
            const bool moving = !(first && still[b]);
            want64[b] = stat[b] == -1 && prec[b] == 1 && moving;
            want32[b] = stat[b] == -1 && prec[b] == 0 && moving;
            nshoot[b] += want64[b] || want32[b];
            any64 = any64 || want64[b];
            any32 = any32 || want32[b];
        }
        if (any64 && want64 != in64) {
            g64.reset();
            pws64.reset(new Workspace(st));
            LM_TRY(make_plan(dim, B, offs, offs_d, tun, *pws64, &pl64, st, &want64, fill));
            in64 = want64;
        }
        if (any32 && want32 != in32) {
            g32.reset();
            pws32.reset(new Workspace(st));
            LM_TRY(make_plan(dim, B, offs, offs_d, tun, *pws32, &pl32, st, &want32, fill));
            in32 = want32;
        }

        // shoot every running problem from (X, p): double-precision ones in place on qd,
        // single-precision ones on qf, copied into qd afterwards
        LM_HIP(hipEventRecord(tm.ev[0], st));
        if (any64 || first) LM_HIP(hipMemcpyAsync(qd, X, m * sizeof(double), hipMemcpyDeviceToDevice, st));
        if (any64) {
            LM_HIP(hipMemcpyAsync(pd, p, m * sizeof(double), hipMemcpyDeviceToDevice, st));
            LM_TRY(batch_shoot_inplace<double>(&p64, pl64, qd, pd, 1.0, o->steps, tun.graph_steps, wd, st, &g64));
        }
        if (any32) {
            LM_HIP((lm::launch_convert<float, double>(pf, p, m, st)));
            LM_HIP(hipMemcpyAsync(qf, xf, m * sizeof(float), hipMemcpyDeviceToDevice, st));
            LM_TRY(batch_shoot_inplace<float>(&p32, pl32, qf, pf, 1.0, o->steps, tun.graph_steps, wf, st, &g32));
            for (int32_t b = 0; b < B; ++b) f32_f[b] = want32[b];
            LM_HIP(hipMemcpyAsync(flags_d + 2 * B, f32_f, B * sizeof(int), hipMemcpyHostToDevice, st));
            LM_HIP(lm::launch_batch_copy_f32_to_f64(qd, qf, dim, ntot, offs_d, flags_d + 2 * B, B, st));
        }
        LM_HIP(hipEventRecord(tm.ev[1], st));
        LM_HIP(lm::launch_batch_maxabsdiff<double>(qd, Y, dim, ntot, offs_d, B, resid_d, st));
        LM_HIP(hipMemcpyAsync(res.data(), resid_d, B * sizeof(double), hipMemcpyDeviceToHost, st));
        LM_HIP(hipStreamSynchronize(st));
        shoot_ms += tm.ms(0, 1);

        // stopping tests (residual below tol in double precision, or in single precision
        // when the match never switches), divergence, iteration limit
        bool any_update = false;
        for (int32_t b = 0; b < B; ++b) {
            upd_f[b] = 0;
            solve_f[b] = 0;
            wide_f[b] = 0;
            const bool shot = want64[b] || want32[b] || (first && still[b] && stat[b] == -1);
            if (!shot) continue;
            info[b].resid_inf = res[b];
            bool hold = false;
            if (!is_finite(res[b])) {
                stat[b] = LM_EDIVERGED;
            } else {
                if (may_switch && prec[b] == 0) {
                    if (res[b] < o->f32_switch) prec[b] = 1;
                    if (res[b] < o->tol || res[b] >= lm::kF32Stall * prevr[b]) {
                        // below tol, or at the single-precision floor: re-shoot the same
                        // momenta in double precision
                        hold = true;
                        prec[b] = 1;
                    }
                }
                prevr[b] = res[b];
                if (!hold && res[b] < o->tol) stat[b] = LM_OK;
                else if (upd[b] >= o->max_iter) stat[b] = LM_ENOTCONV;
                else if (!hold) upd_f[b] = 1;
            }
            if (stat[b] != -1 && q1_out) {
                const int64_t nb = offs[b + 1] - offs[b];
                for (int c = 0; c < dim; ++c)
                    LM_HIP(hipMemcpyAsync(q1_out + c * ntot + offs[b], qd + c * ntot + offs[b], nb * sizeof(double),
                                          hipMemcpyDeviceToDevice, st));
            }
            if (upd_f[b]) {
                any_update = true;
                solve_f[b] = (offs[b + 1] - offs[b]) <= wide_min;
                wide_f[b] = !solve_f[b];
            }
        }
        first = false;
        bool running = false;
        for (int32_t b = 0; b < B; ++b) running = running || stat[b] == -1;
        if (!running) break;
        if (!any_update) continue;   // only re-shoots in double precision this round

        // p_b <- p_b + h (K_b + tau I)^{-1} (Y_b - q_b(1)) for the problems that update
        LM_HIP(hipEventRecord(tm.ev[2], st));
        LM_HIP(lm::launch_sub(e, Y, qd, m, st));
        LM_HIP(hipMemcpyAsync(flags_d, flags.data(), 2 * B * sizeof(int), hipMemcpyHostToDevice, st));
        LM_HIP(hipMemcpyAsync(flags_d + 3 * B, wide_f, B * sizeof(int), hipMemcpyHostToDevice, st));
        if (witems) {
            // disjoint problems: the one-workgroup solves on the side stream, the wide sweeps here
            LM_TRY(fj.fork(st));
            LM_HIP(lm::launch_batch_dense_solve(L, loff_d, Linv, ioff_d, offs_d, B, dim, ntot, e, flags_d + B, fj.s));
            LM_HIP(lm::launch_batch_wide_solve(L, loff_d, Linv, ioff_d, offs_d, dim, ntot, e, flags_d + 3 * B, witems,
                                               wplan, st));
            LM_TRY(fj.join(st));
        } else {
            LM_HIP(lm::launch_batch_dense_solve(L, loff_d, Linv, ioff_d, offs_d, B, dim, ntot, e, flags_d + B, st));
        }
        LM_HIP(lm::launch_batch_axpy(p, e, o->h, dim, ntot, offs_d, flags_d, B, st));
        LM_HIP(hipEventRecord(tm.ev[3], st));
        // the host flags are rewritten next iteration: wait until the uploads are consumed
        LM_HIP(hipEventSynchronize(tm.ev[3]));
        solve_ms += tm.ms(2, 3);
        for (int32_t b = 0; b < B; ++b) upd[b] += upd_f[b];
    }
    if (q1_out) {
        // a problem with a singular K is never shot: report q(1) = X for it
        for (int32_t b = 0; b < B; ++b) {
            if (stat[b] != LM_ESINGULAR) continue;
            const int64_t nb = offs[b + 1] - offs[b];
            for (int c = 0; c < dim; ++c)
                LM_HIP(hipMemcpyAsync(q1_out + c * ntot + offs[b], X + c * ntot + offs[b], nb * sizeof(double),
                                      hipMemcpyDeviceToDevice, st));
        }
    }

    // H_b = 1/2 sum (p_b . K(X_b) p_b): velocities of the batch at (X, p), then per-problem dots
    {
        Workspace hws(st);
        BatchPlan pl;
        LM_TRY(make_plan(dim, B, offs, offs_d, tun, hws, &pl, st));
        // H is the kernel form alone (equation "H"): the inexact advection weight tau is not
        // part of it, so the velocities are summed with tau = 0
        lm::EpiArgs<double> ev{};
        ev.kind = lm::EPI_STORE;
        ev.tau = 0.0;
        ev.in_p = p;
        ev.out_q = e;
        ev.out_p = qd;   // forces are not needed; written to scratch
        LM_TRY(batch_eval<double>(&p64, pl, X, p, ev, st));
        LM_HIP(lm::launch_batch_dot(p, e, dim, ntot, offs_d, B, resid_d, st));
        std::vector<double> hb((size_t)B);
        LM_HIP(hipMemcpyAsync(hb.data(), resid_d, B * sizeof(double), hipMemcpyDeviceToHost, st));
        LM_HIP(hipStreamSynchronize(st));
        for (int32_t b = 0; b < B; ++b) info[b].H = 0.5 * hb[b];
    }

    lm_status result = LM_OK;
    const lm_status order[3] = {LM_EDIVERGED, LM_ESINGULAR, LM_ENOTCONV};
    for (lm_status s : order)
        for (int32_t b = 0; b < B && result == LM_OK; ++b)
            if (stat[b] == s) result = s;
    for (int32_t b = 0; b < B; ++b) {
        info[b].iters = upd[b];
        info[b].cg_iters = 0;
        info[b].shoot_ms = shoot_ms;
        info[b].solve_ms = solve_ms;
        info[b].factor_ms = factor_ms;
        info[b].shoots = nshoot[b];
        if (stat[b] == LM_ESINGULAR) info[b].resid_inf = NAN;
        if (status) status[b] = stat[b];
    }
    if (result != LM_OK) {
        int32_t nbad = 0;
        for (int32_t b = 0; b < B; ++b) nbad += stat[b] != LM_OK;
        fail(result, "%d of %d problems did not converge (per-problem status in status[])", nbad, B);
    }
    return result;
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================

extern "C" {

lm_status lm_batch_default_tuning(int32_t B, const int64_t* offs, lm_batch_tuning* out)
{
    if (!out) return fail(LM_EINVAL, "out is NULL");
    int64_t ntot;
    return resolve_tuning(nullptr, B, offs, out, &ntot);
}

lm_status lm_batch_autotune(const lm_params* prm, int32_t B, const int64_t* offs, const void* q, const void* p,
                            lm_batch_tuning* out, void* stream)
{
    LM_TRY(check_batch_params(prm));
    if (!q || !p || !out) return fail(LM_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F32)
        return autotune_t<float>(prm, B, offs, (const float*)q, (const float*)p, out, st);
    return autotune_t<double>(prm, B, offs, (const double*)q, (const double*)p, out, st);
}

lm_status lm_rhs_batched(const lm_params* prm, int32_t B, const int64_t* offs, const void* q, const void* p, void* dq,
                         void* dp, const lm_batch_tuning* tuning, void* stream)
{
    LM_TRY(check_batch_params(prm));
    if (!q || !p || !dq || !dp) return fail(LM_EINVAL, "NULL buffer");
    if (dq == q || dq == p || dp == q || dp == p || dq == dp) return fail(LM_EINVAL, "outputs must not alias inputs");
    lm_batch_tuning t;
    int64_t ntot;
    LM_TRY(resolve_tuning(tuning, B, offs, &t, &ntot));
    hipStream_t st = (hipStream_t)stream;
    Workspace ws(st);
    int64_t* offs_d;
    LM_TRY(upload_offs(B, offs, ws, &offs_d, st));
    BatchPlan pl;
    LM_TRY(make_plan(prm->dim, B, offs, offs_d, t, ws, &pl, st));
    if (prm->dtype == LM_F32)
        return batch_rhs<float>(prm, pl, (const float*)q, (const float*)p, (float*)dq, (float*)dp, st);
    return batch_rhs<double>(prm, pl, (const double*)q, (const double*)p, (double*)dq, (double*)dp, st);
}

lm_status lm_shoot_batched(const lm_params* prm, int32_t B, const int64_t* offs, const void* q0, const void* p0,
                           double t1, int32_t steps, void* q1, void* p1, const lm_batch_tuning* tuning, void* stream)
{
    LM_TRY(check_batch_params(prm));
    if (!q0 || !p0 || !q1 || !p1) return fail(LM_EINVAL, "NULL buffer");
    if (steps < 1) return fail(LM_EINVAL, "steps must be >= 1");
    if (!is_finite(t1)) return fail(LM_EINVAL, "t1 must be finite");
    lm_batch_tuning t;
    int64_t ntot;
    LM_TRY(resolve_tuning(tuning, B, offs, &t, &ntot));
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F32)
        return shoot_batched_t<float>(prm, B, offs, (const float*)q0, (const float*)p0, t1, steps, (float*)q1,
                                      (float*)p1, t, st);
    return shoot_batched_t<double>(prm, B, offs, (const double*)q0, (const double*)p0, t1, steps, (double*)q1,
                                   (double*)p1, t, st);
}

lm_status lm_feedback_match_batched(const lm_params* prm, const lm_match_opts* o, int32_t B, const int64_t* offs,
                                    const double* X, const double* Y, double* p0, double* q1, lm_match_info* info,
                                    int32_t* status, const lm_batch_tuning* tuning, void* stream)
{
    LM_TRY(check_batch_params(prm));
    if (!o) return fail(LM_EINVAL, "opts is NULL");
    if (!X || !Y || !p0 || !info) return fail(LM_EINVAL, "NULL argument");
    if (!(o->h > 0.0) || !is_finite(o->h)) return fail(LM_EINVAL, "h must be positive and finite");
    if (!(o->tol > 0.0) || !is_finite(o->tol)) return fail(LM_EINVAL, "tol must be positive and finite");
    if (o->max_iter < 0) return fail(LM_EINVAL, "max_iter must be >= 0");
    if (o->steps < 1) return fail(LM_EINVAL, "steps must be >= 1");
    if (o->stop_rule != 0) return fail(LM_EUNSUPPORTED, "batched matching supports stop_rule 0 only");
    lm_batch_tuning t;
    int64_t ntot;
    LM_TRY(resolve_tuning(tuning, B, offs, &t, &ntot));
    return match_batched(prm, o, B, offs, X, Y, p0, q1, info, status, t, (hipStream_t)stream);
}

}  // extern "C"
