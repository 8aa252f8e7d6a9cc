// lm_api.hip -- host side of the C ABI declared in include/liblm.h.
//
// Argument checks, stream-ordered workspace, and the loops that sequence the kernels of
// lm_kernels.hip: the Runge-Kutta stage loop of a shoot, the conjugate-gradient K-solve and
// Algorithm 1's feedback loop.  No arithmetic of the method runs on the host: the host only
// decides what to launch next and reads back the scalars that decide it (the residual of
// each shoot, the CG residual norms).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lm_host.h"
#include "lm_internal.h"

namespace lmh {

namespace {
thread_local std::string g_err;
}

lm_status fail(lm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

lm_status fail_hip(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory) return fail(LM_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(LM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

lm_status check_params(const lm_params* prm)
{
    if (!prm) return fail(LM_EINVAL, "params is NULL");
    if (prm->dim != 2 && prm->dim != 3) return fail(LM_EINVAL, "dim must be 2 or 3 (got %d)", prm->dim);
    if (prm->kernel != LM_KERNEL_CONON && prm->kernel != LM_KERNEL_GAUSS)
        return fail(LM_EINVAL, "unknown kernel %d", prm->kernel);
    if (prm->dtype != LM_F64 && prm->dtype != LM_F32) return fail(LM_EINVAL, "unknown dtype %d", prm->dtype);
    if (prm->flags != 0) return fail(LM_EINVAL, "flags must be 0");
    if (!(prm->sigma > 0.0) || !is_finite(prm->sigma)) return fail(LM_EINVAL, "sigma must be positive and finite");
    if (!(prm->tau >= 0.0) || !is_finite(prm->tau)) return fail(LM_EINVAL, "tau must be >= 0 and finite");
    if (!(prm->cutoff >= 0.0) || !is_finite(prm->cutoff)) return fail(LM_EINVAL, "cutoff must be >= 0 and finite");
    return LM_OK;
}

lm_status check_n(int64_t n, const char* name)
{
    if (n < 1 || n > kMaxN) return fail(LM_EINVAL, "%s must be in [1, 2^34] (got %lld)", name, (long long)n);
    return LM_OK;
}

void kernel_scales(const lm_params* prm, double* kq, double* wscale)
{
    const double s = prm->sigma;
    if (prm->kernel == LM_KERNEL_CONON) {
        *kq = -kLog2e / s;
        *wscale = 1.0 / s;
    } else {
        *kq = -kLog2e / (s * s);
        *wscale = 2.0 / (s * s);
    }
}

}  // namespace lmh

namespace {

using namespace lmh;

// Cutoff mode: tile boxes of the sources and of the targets (the same buffer when the
// targets are the sources) and the squared radius.  box_s == nullptr means every pair.
struct Cut {
    const double* box_s = nullptr;
    const double* box_t = nullptr;
    double rc2 = 0.0;
};

// One evaluation of the pair sums with targets (qt, pt) [nt] and sources (qs, ps) [ns].
// tscale > 0: the sources are in the exponent's units and the targets are multiplied by
// tscale (see PairArgs).
template <class T>
lm_status pair_eval(const lm_params* prm, bool force, const T* qs, const T* ps, int64_t ns, const T* qt,
                    const T* pt, int64_t nt, const lm::EpiArgs<T>& epi, double* part, hipStream_t st,
                    const Cut& cut = Cut(), double tscale = 0.0)
{
    const bool sym_ok = qs == qt && ps == pt && ns == nt;
    lm::PairPlan pl = lm::plan_pair(nt, ns, cut.box_s != nullptr, sym_ok, sizeof(T) == 4 ? lm::SYM_F32 : lm::SYM_F64);
    lm::PairArgs<T> a{};
    a.qs = qs;
    a.ps = ps;
    a.qt = qt;
    a.pt = pt;
    a.nt = nt;
    a.ns = ns;
    a.jchunk = pl.jchunk;
    kernel_scales(prm, &a.kq, &a.wscale);
    a.tscale = tscale;
    if (tscale > 0.0 && prm->kernel != LM_KERNEL_CONON) a.wscale /= std::sqrt(-a.kq);
    a.part = reinterpret_cast<T*>(part);   // the workspace is sized in doubles; slots are T
    a.box_s = cut.box_s;
    a.box_t = cut.box_t;
    a.rc2 = cut.rc2;
    a.epi = epi;
    LM_HIP(lm::launch_pair<T>(prm->dim, prm->kernel, force, a, pl, st));
    return LM_OK;
}

// Workspace of the split partial sums: enough for either kernel that pair_eval may choose.
int64_t part_elems(const lm_params* prm, int64_t nt, int64_t ns)
{
    const lm::PairPlan pl = lm::plan_pair(nt, ns, false);
    int64_t m = pl.nsplit > 1 ? (int64_t)pl.nsplit * 2 * prm->dim * nt : 1;
    if (nt == ns) {
        // the symmetric kernel's slots under any setting of LM_SYM (forced or by size), and its
        // superblock-pair flags in tile-skipping mode
        for (int cut = 0; cut < 2; ++cut) {
            const lm::SymPlan sp = lm::plan_sym(nt, true, prm->dtype == LM_F32 ? lm::SYM_F32 : lm::SYM_F64, cut == 1);
            if (sp.waves > 0) {
                const int64_t ms = (sp.nsb + 1) * 2 * prm->dim * nt + lm::sym_flag_elems(sp.nsb);
                if (ms > m) m = ms;
            }
        }
    }
    return m;
}

// Workspace of a VJP evaluation: the interleaved source copy, then the partial sums of either
// VJP kernel (and of the forward sums, which share the buffer in the adjoint).
int64_t vjp_part_elems(const lm_params* prm, int64_t n)
{
    int64_t m = part_elems(prm, n, n);
    const lm::SymPlan sp = lm::plan_sym(n, true, lm::SYM_VJP);
    if (sp.waves > 0 && (sp.nsb + 1) * 2 * prm->dim * n > m) m = (sp.nsb + 1) * 2 * prm->dim * n;
    return 4 * (int64_t)prm->dim * n + m;
}

// Passive points carried along by a shoot (equation "u"): positions x (dim, m), advanced in
// place, with stage buffers ax, bx and the RK4 running sum cx (dim*m T each).  box (cutoff
// mode, tiles_of(m)*8 doubles) receives the tile boxes of every stage's points.
template <class T>
struct Points {
    int64_t m = 0;
    T* x = nullptr;
    T *ax = nullptr, *bx = nullptr, *cx = nullptr;
    double* box = nullptr;
};

// RK4 shoot of (q, p) in place over [0, t1] with `steps` steps.  a*, b*: stage buffers, c*:
// the RK4 running sum (dim*n T each); part: the split workspace.  box (non-null in cutoff
// mode, tiles_of(n)*8 doubles) receives the tile boxes of every stage input.  pts
// (nullable): points advected by the velocity field of every stage's particles; each stage
// evaluates their velocities before the particles' own launch overwrites that stage's
// inputs' successor.
template <class T>
lm_status shoot_inplace(const lm_params* prm, int64_t n, T* q, T* p, double t1, int32_t steps, T* aq, T* ap,
                        T* bq, T* bp, T* cq, T* cp, double* part, hipStream_t st, double* box = nullptr,
                        const Points<T>* pts = nullptr)
{
    const double dt = t1 / steps;
    if (!box && !pts && lm::small_path(n, prm->dim, sizeof(T) == 4)) {
        // the whole shoot in one launch (one workgroup holds the problem)
        lm::SmallShootArgs<T> a{};
        a.q = q;
        a.p = p;
        a.ntot = n;
        a.offs = nullptr;
        a.dt = dt;
        a.steps = steps;
        kernel_scales(prm, &a.kq, &a.wscale);
        a.tau = prm->tau;
        LM_HIP(lm::launch_small_shoot<T>(prm->dim, prm->kernel, a, 1, st));
        return LM_OK;
    }
    lm::EpiArgs<T> e{};
    e.dt = dt;
    e.tau = prm->tau;
    e.base_q = q;
    e.base_p = p;
    e.acc_q = cq;
    e.acc_p = cp;
    // With one-sided pair sums and no tile skipping the stages run on positions in the
    // exponent's units (ks q), which takes a multiply out of every pair: the first stage
    // reads ks y from B (written here, then by each step's last stage, when B is free), and
    // the other stages' position outputs are written scaled.  The state y stays unscaled.
    double kq0, ws0;
    kernel_scales(prm, &kq0, &ws0);
    const double ks = prm->kernel == LM_KERNEL_CONON ? -kq0 : std::sqrt(-kq0);
    const bool pre = !box && lm::plan_pair(n, n, false, true, sizeof(T) == 4 ? lm::SYM_F32 : lm::SYM_F64).sym_waves == 0;
    if (pre) {
        e.qscale = ks;
        e.out_qs = bq;
        LM_HIP(lm::launch_scaled_copy<T>(bq, q, ks, (int64_t)prm->dim * n, st));
    }
    Cut cut;
    if (box) {
        cut.box_s = cut.box_t = box;
        cut.rc2 = prm->cutoff * prm->cutoff;
    }
    lm::EpiArgs<T> ex{};
    Cut xcut;
    if (pts) {
        ex.dt = dt;
        ex.tau = 0.0;
        ex.base_q = pts->x;
        ex.acc_q = pts->cx;
        if (box) {
            xcut.box_s = box;
            xcut.box_t = pts->box;
            xcut.rc2 = cut.rc2;
        }
    }
    for (int32_t s = 0; s < steps; ++s) {
        // stage 1: input y, output A ; stage 2: A -> B ; stage 3: B -> A ; stage 4: A -> y
        const T* in_q[4] = {pre ? bq : q, aq, bq, aq};
        const T* in_p[4] = {p, ap, bp, ap};
        T* out_q[4] = {aq, bq, aq, q};
        T* out_p[4] = {ap, bp, ap, p};
        for (int k = 0; k < 4; ++k) {
            e.kind = lm::EPI_RK1 + k;
            e.in_p = in_p[k];
            e.out_q = out_q[k];
            e.out_p = out_p[k];
            if (box) LM_HIP(lm::launch_tile_boxes<T>(prm->dim, in_q[k], n, box, st));
            if (pts) {
                // the points' stage on the same buffer rotation: x -> A -> B -> A -> x
                const T* in_x[4] = {pts->x, pts->ax, pts->bx, pts->ax};
                T* out_x[4] = {pts->ax, pts->bx, pts->ax, pts->x};
                ex.kind = lm::EPI_RK1 + k;
                ex.out_q = out_x[k];
                if (box) LM_HIP(lm::launch_tile_boxes<T>(prm->dim, in_x[k], pts->m, pts->box, st));
                LM_TRY(pair_eval<T>(prm, false, in_q[k], in_p[k], n, in_x[k], (const T*)nullptr, pts->m, ex, part, st,
                                    xcut, pre ? ks : 0.0));
            }
            LM_TRY(pair_eval<T>(prm, true, in_q[k], in_p[k], n, in_q[k], in_p[k], n, e, part, st, cut,
                                pre ? 1.0 : 0.0));
        }
    }
    return LM_OK;
}

// Spatial order of a point set for the cutoff mode: perm (n indices) sorts the points by
// the Morton code of their position.
struct Ordering {
    int64_t* perm = nullptr;
    double* box = nullptr;    // tile boxes, reused by the shoot for its stage boxes
    lm_status alloc(Workspace& ws, int64_t n);
    template <class T>
    lm_status compute(int dim, const T* q, int64_t n, Workspace& ws, hipStream_t st)
    {
        double* gbox;
        uint64_t* keys;
        LM_TRY(ws.get(&gbox, 8));
        LM_TRY(ws.get(&keys, lm::sort_pad(n)));
        LM_HIP(lm::launch_morton_order<T>(dim, q, n, box, gbox, keys, perm, st));
        return LM_OK;
    }
};

lm_status Ordering::alloc(Workspace& ws, int64_t n)
{
    LM_TRY(ws.get(&perm, n));
    LM_TRY(ws.get(&box, lm::tiles_of(n) * 8));
    return LM_OK;
}

constexpr int64_t kMaxCutN = ((int64_t)1 << 31) - 1;

template <class T>
lm_status shoot_t(const lm_params* prm, int64_t n, const T* q0, const T* p0, double t1, int32_t steps, T* q1,
                  T* p1, hipStream_t st)
{
    const int64_t m = (int64_t)prm->dim * n;
    Workspace ws(st);
    T *aq, *ap, *bq, *bp, *cq, *cp;
    double* part;
    LM_TRY(ws.get(&aq, m));
    LM_TRY(ws.get(&ap, m));
    LM_TRY(ws.get(&bq, m));
    LM_TRY(ws.get(&bp, m));
    LM_TRY(ws.get(&cq, m));
    LM_TRY(ws.get(&cp, m));
    LM_TRY(ws.get(&part, part_elems(prm, n, n)));
    if (prm->cutoff > 0.0) {
        // shoot in Morton order so that tiles are compact, then scatter back
        if (n > kMaxCutN) return fail(LM_EINVAL, "cutoff mode needs n < 2^31");
        Ordering ord;
        LM_TRY(ord.alloc(ws, n));
        LM_TRY(ord.compute<T>(prm->dim, q0, n, ws, st));
        T *sq, *sp;
        LM_TRY(ws.get(&sq, m));
        LM_TRY(ws.get(&sp, m));
        LM_HIP((lm::launch_permute<T, T>(sq, q0, ord.perm, n, prm->dim, false, st)));
        LM_HIP((lm::launch_permute<T, T>(sp, p0, ord.perm, n, prm->dim, false, st)));
        LM_TRY(shoot_inplace<T>(prm, n, sq, sp, t1, steps, aq, ap, bq, bp, cq, cp, part, st, ord.box));
        LM_HIP((lm::launch_permute<T, T>(q1, sq, ord.perm, n, prm->dim, true, st)));
        LM_HIP((lm::launch_permute<T, T>(p1, sp, ord.perm, n, prm->dim, true, st)));
        return LM_OK;
    }
    if (q1 != q0) LM_HIP(hipMemcpyAsync(q1, q0, m * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (p1 != p0) LM_HIP(hipMemcpyAsync(p1, p0, m * sizeof(T), hipMemcpyDeviceToDevice, st));
    return shoot_inplace<T>(prm, n, q1, p1, t1, steps, aq, ap, bq, bp, cq, cp, part, st);
}

// Shoot of (q0, p0) over [0, t1] carrying the points x0 (dim, m) along: results to q1, p1 (each
// nullable: then kept in workspace) and x1 (may alias x0).
template <class T>
lm_status flow_t(const lm_params* prm, int64_t n, const T* q0, const T* p0, int64_t m, const T* x0, double t1,
                 int32_t steps, T* q1, T* p1, T* x1, hipStream_t st)
{
    const int64_t mq = (int64_t)prm->dim * n, mx = (int64_t)prm->dim * m;
    Workspace ws(st);
    T *aq, *ap, *bq, *bp, *cq, *cp, *sq, *sp;
    double* part;
    Points<T> pts;
    pts.m = m;
    pts.x = x1;
    LM_TRY(ws.get(&aq, mq));
    LM_TRY(ws.get(&ap, mq));
    LM_TRY(ws.get(&bq, mq));
    LM_TRY(ws.get(&bp, mq));
    LM_TRY(ws.get(&cq, mq));
    LM_TRY(ws.get(&cp, mq));
    LM_TRY(ws.get(&pts.ax, mx));
    LM_TRY(ws.get(&pts.bx, mx));
    LM_TRY(ws.get(&pts.cx, mx));
    const int64_t pe = std::max(part_elems(prm, n, n), part_elems(prm, m, n));
    LM_TRY(ws.get(&part, pe));
    const bool order = prm->cutoff > 0.0;
    Ordering ord;
    if (order) {
        if (n > kMaxCutN || m > kMaxCutN) return fail(LM_EINVAL, "cutoff mode needs n, m < 2^31");
        LM_TRY(ord.alloc(ws, n));
        LM_TRY(ws.get(&pts.box, lm::tiles_of(m) * 8));
    }
    // the particles evolve in sq, sp: q1/p1 themselves unless they are absent or the cutoff
    // mode keeps the particles in Morton order
    if (order || !q1) LM_TRY(ws.get(&sq, mq)); else sq = q1;
    if (order || !p1) LM_TRY(ws.get(&sp, mq)); else sp = p1;
    if (x1 != x0) LM_HIP(hipMemcpyAsync(x1, x0, mx * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (order) {
        LM_TRY(ord.compute<T>(prm->dim, q0, n, ws, st));
        LM_HIP((lm::launch_permute<T, T>(sq, q0, ord.perm, n, prm->dim, false, st)));
        LM_HIP((lm::launch_permute<T, T>(sp, p0, ord.perm, n, prm->dim, false, st)));
    } else {
        if (sq != q0) LM_HIP(hipMemcpyAsync(sq, q0, mq * sizeof(T), hipMemcpyDeviceToDevice, st));
        if (sp != p0) LM_HIP(hipMemcpyAsync(sp, p0, mq * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    LM_TRY(shoot_inplace<T>(prm, n, sq, sp, t1, steps, aq, ap, bq, bp, cq, cp, part, st, order ? ord.box : nullptr,
                            &pts));
    if (order) {
        if (q1) LM_HIP((lm::launch_permute<T, T>(q1, sq, ord.perm, n, prm->dim, true, st)));
        if (p1) LM_HIP((lm::launch_permute<T, T>(p1, sp, ord.perm, n, prm->dim, true, st)));
    }
    return LM_OK;
}

// Hamiltonian in double: H = 1/2 sum_c p_c . (K p)_c.  q, p double.
lm_status hamiltonian_f64(const lm_params* prm, int64_t n, const double* q, const double* p, double* H,
                          hipStream_t st)
{
    const int dim = prm->dim;
    Workspace ws(st);
    double *v, *part, *red, *dots;
    LM_TRY(ws.get(&v, dim * n));
    LM_TRY(ws.get(&part, part_elems(prm, n, n)));
    LM_TRY(ws.get(&red, (int64_t)lm::reduce_blocks(n) * dim));
    LM_TRY(ws.get(&dots, dim));
    lm::EpiArgs<double> e{};
    e.kind = lm::EPI_STORE;
    e.tau = 0.0;
    e.out_q = v;
    LM_TRY(pair_eval<double>(prm, false, q, p, n, q, p, n, e, part, st));
    LM_HIP(lm::launch_dots(p, v, n, dim, red, dots, st));
    double hd[3] = {0, 0, 0};
    LM_HIP(hipMemcpyAsync(hd, dots, dim * sizeof(double), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (int c = 0; c < dim; ++c) s += hd[c];
    *H = 0.5 * s;
    return LM_OK;
}

// CG for (K(X) + tau I) x_c = b_c, all components in lockstep.  Buffers in `cg` are dim*n
// doubles each (r, p, Ap) plus scalars; `part` is the pair-split workspace.
struct CgBuffers {
    double *r, *p, *ap, *red, *rr, *rr_new, *pap, *bb;
};

lm_status cg_alloc(Workspace& ws, const lm_params* prm, int64_t n, CgBuffers* b)
{
    const int64_t m = (int64_t)prm->dim * n;
    LM_TRY(ws.get(&b->r, m));
    LM_TRY(ws.get(&b->p, m));
    LM_TRY(ws.get(&b->ap, m));
    LM_TRY(ws.get(&b->red, (int64_t)lm::reduce_blocks(n) * prm->dim));
    LM_TRY(ws.get(&b->rr, 3));
    LM_TRY(ws.get(&b->rr_new, 3));
    LM_TRY(ws.get(&b->pap, 3));
    LM_TRY(ws.get(&b->bb, 3));
    return LM_OK;
}

lm_status ksolve_impl(const lm_params* prm, int64_t n, const double* X, const double* b, double* x, double rtol,
                      int32_t max_iter, int32_t* iters_out, CgBuffers& cg, double* part, hipStream_t st)
{
    const int dim = prm->dim;
    const int64_t m = (int64_t)dim * n;
    // r = b ; x = 0 ; p = r ; rr = bb = r.r
    LM_HIP(hipMemcpyAsync(cg.r, b, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(lm::launch_zero(x, m, st));
    LM_HIP(hipMemcpyAsync(cg.p, cg.r, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(lm::launch_dots(cg.r, cg.r, n, dim, cg.red, cg.rr, st));
    LM_HIP(hipMemcpyAsync(cg.bb, cg.rr, dim * sizeof(double), hipMemcpyDeviceToDevice, st));
    double bb[3] = {0, 0, 0}, h[6];
    LM_HIP(hipMemcpyAsync(bb, cg.bb, dim * sizeof(double), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < dim; ++c)
        if (!is_finite(bb[c])) return fail(LM_EDIVERGED, "non-finite right-hand side in the K-solve");

    lm::EpiArgs<double> e{};
    e.kind = lm::EPI_STORE;
    e.tau = prm->tau;
    e.out_q = cg.ap;
    int32_t it = 0;
    bool done = true;
    for (int c = 0; c < dim; ++c) done = done && (bb[c] == 0.0);
    while (!done) {
        if (it >= max_iter) {
            if (iters_out) *iters_out = it;
            return fail(LM_ENOTCONV, "K-solve: %d CG iterations without reaching rtol %.3g", it, rtol);
        }
        // Ap = (K + tau I) p
        e.in_p = cg.p;
        LM_TRY(pair_eval<double>(prm, false, X, cg.p, n, X, cg.p, n, e, part, st));
        LM_HIP(lm::launch_dots(cg.p, cg.ap, n, dim, cg.red, cg.pap, st));
        LM_HIP(lm::launch_cg_update_xr(x, cg.r, cg.p, cg.ap, cg.rr, cg.pap, n, dim, st));
        LM_HIP(lm::launch_dots(cg.r, cg.r, n, dim, cg.red, cg.rr_new, st));
        LM_HIP(lm::launch_cg_update_p(cg.p, cg.r, cg.rr_new, cg.rr, n, dim, st));
        LM_HIP(hipMemcpyAsync(h, cg.rr_new, dim * sizeof(double), hipMemcpyDeviceToHost, st));
        LM_HIP(hipMemcpyAsync(h + 3, cg.pap, dim * sizeof(double), hipMemcpyDeviceToHost, st));
        std::swap(cg.rr, cg.rr_new);
        LM_HIP(hipStreamSynchronize(st));
        ++it;
        done = true;
        for (int c = 0; c < dim; ++c) {
            const double rrc = h[c], papc = h[3 + c];
            if (!is_finite(rrc) || !is_finite(papc)) {
                if (iters_out) *iters_out = it;
                return fail(LM_ESINGULAR, "K-solve: non-finite CG scalars (K not positive definite?)");
            }
            if (bb[c] > 0.0 && !(papc > 0.0) && rrc > rtol * rtol * bb[c]) {
                if (iters_out) *iters_out = it;
                return fail(LM_ESINGULAR, "K-solve: non-positive curvature p.Kp = %g", papc);
            }
            if (!(rrc <= rtol * rtol * bb[c])) done = false;
        }
    }
    if (iters_out) *iters_out = it;
    return LM_OK;
}

// Dense Cholesky factor of K(X) + tau I (see lm_dense.hip).  With W set, the solves run the
// superblock sweeps (W: the diagonal superblocks' inverses; scratch: their work vectors).
struct DenseFactor {
    double* L = nullptr;
    double* Linv = nullptr;
    double* W = nullptr;
    double* scratch = nullptr;
    int* info = nullptr;
    int64_t n = 0;
};

// Superblock sweeps for an n-point factor: LM_DENSE_SUPER (0/1) overrides the default (on
// when n spans more than one superblock of 8 x 128 rows).
bool use_super(int64_t n)
{
    if (const char* e = std::getenv("LM_DENSE_SUPER")) return e[0] == '1';
    return lm::dense_super_default(n);
}

// Whether the dense factor of an n-point problem fits in half the free device memory.
bool dense_fits(int64_t n)
{
    if (n >= lm::kDenseMaxN) return false;
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return false;
    double need = 8.0 * (double)n * (double)n + 8.0 * (double)lm::dense_linv_elems(n);
    if (use_super(n))
        need += 8.0 * (double)(lm::dense_super_elems(n) + lm::dense_solve_scratch_elems(n));
    need += 4.0 * (double)lm::dense_panel_f32_elems(n);   // a single-precision factor's panel copy
    return need <= 0.5 * (double)freeb;
}

// f32_update: the trailing updates multiply in single precision (for solves that only steer a
// match with single-precision shoots), staging a float copy of each update's operand columns;
// LM_FACTOR_F32 (0/1) overrides the choice and LM_FACTOR_F32_PANEL=0 stages from the FP64
// matrix instead (the same result; for comparison).
lm_status dense_factor(const lm_params* prm, int64_t n, const double* X, Workspace& ws, DenseFactor* f,
                       hipStream_t st, bool f32_update = false)
{
    if (const char* e = std::getenv("LM_FACTOR_F32")) f32_update = e[0] == '1';
    float* panel = nullptr;
    if (f32_update) {
        const char* e = std::getenv("LM_FACTOR_F32_PANEL");
        if (!(e && e[0] == '0')) LM_TRY(ws.get(&panel, lm::dense_panel_f32_elems(n)));
    }
    f->n = n;
    LM_TRY(ws.get(&f->L, n * n));
    LM_TRY(ws.get(&f->Linv, lm::dense_linv_elems(n)));
    LM_TRY(ws.get(&f->info, 1));
    if (use_super(n)) {
        LM_TRY(ws.get(&f->W, lm::dense_super_elems(n)));
        LM_TRY(ws.get(&f->scratch, lm::dense_solve_scratch_elems(n)));
    }
    double kq, wscale;
    kernel_scales(prm, &kq, &wscale);
    LM_HIP(lm::launch_dense_factor(prm->dim, prm->kernel, kq, prm->tau, X, n, f->L, f->Linv, f->info, st,
                                   f32_update, panel));
    if (f->W) LM_HIP(lm::launch_dense_super(f->L, f->Linv, n, f->W, st));
    int info = 0;
    LM_HIP(hipMemcpyAsync(&info, f->info, sizeof(int), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    if (info != 0)
        return fail(LM_ESINGULAR, "K(X) is not numerically positive definite (Cholesky pivot %d)", info);
    return LM_OK;
}

// x = (K + tau I)^{-1} b with the dense factor (x may alias b).
lm_status dense_solve(const DenseFactor& f, int dim, const double* b, double* x, hipStream_t st)
{
    if (x != b) LM_HIP(hipMemcpyAsync(x, b, (size_t)dim * f.n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (f.W)
        LM_HIP(lm::launch_dense_solve_super(f.L, f.Linv, f.W, f.n, dim, x, f.n, f.scratch, st));
    else
        LM_HIP(lm::launch_dense_solve(f.L, f.Linv, f.n, dim, x, f.n, st));
    return LM_OK;
}

// Resolves LM_SOLVE_AUTO.
lm_status pick_solver(int32_t solver, int64_t n, bool* dense)
{
    if (solver == LM_SOLVE_CG) {
        *dense = false;
    } else if (solver == LM_SOLVE_DENSE) {
        if (!dense_fits(n)) return fail(LM_ENOMEM, "dense K factor of n = %lld does not fit", (long long)n);
        *dense = true;
    } else if (solver == LM_SOLVE_AUTO) {
        *dense = dense_fits(n);
    } else {
        return fail(LM_EINVAL, "unknown solver %d", solver);
    }
    return LM_OK;
}

// Right-hand side in the caller's order; in cutoff mode the tiles are 64 consecutive points
// of that order.
template <class T>
lm_status rhs_t(const lm_params* prm, int64_t n, const T* q, const T* p, T* dq, T* dp, hipStream_t st)
{
    Workspace ws(st);
    double* part;
    LM_TRY(ws.get(&part, part_elems(prm, n, n)));
    Cut cut;
    if (prm->cutoff > 0.0) {
        double* box;
        LM_TRY(ws.get(&box, lm::tiles_of(n) * 8));
        LM_HIP(lm::launch_tile_boxes<T>(prm->dim, q, n, box, st));
        cut.box_s = cut.box_t = box;
        cut.rc2 = prm->cutoff * prm->cutoff;
    }
    lm::EpiArgs<T> e{};
    e.kind = lm::EPI_STORE;
    e.tau = prm->tau;
    e.in_p = p;
    e.out_q = dq;
    e.out_p = dp;
    return pair_eval<T>(prm, true, q, p, n, q, p, n, e, part, st, cut);
}

template <class T>
lm_status velocity_t(const lm_params* prm, int64_t n, const T* q, const T* p, int64_t m, const T* x, T* u,
                     hipStream_t st)
{
    Workspace ws(st);
    double* part;
    LM_TRY(ws.get(&part, part_elems(prm, m, n)));
    Cut cut;
    if (prm->cutoff > 0.0) {
        double *bs, *bt;
        LM_TRY(ws.get(&bs, lm::tiles_of(n) * 8));
        LM_TRY(ws.get(&bt, lm::tiles_of(m) * 8));
        LM_HIP(lm::launch_tile_boxes<T>(prm->dim, q, n, bs, st));
        LM_HIP(lm::launch_tile_boxes<T>(prm->dim, x, m, bt, st));
        cut.box_s = bs;
        cut.box_t = bt;
        cut.rc2 = prm->cutoff * prm->cutoff;
    }
    lm::EpiArgs<T> e{};
    e.kind = lm::EPI_STORE;
    e.tau = 0.0;
    e.out_q = u;
    return pair_eval<T>(prm, false, q, p, n, x, (const T*)nullptr, m, e, part, st, cut);
}

lm_status check_match_args(const lm_match_opts* o, const double* X, const double* Y, const double* p0)
{
    if (!o) return fail(LM_EINVAL, "opts is NULL");
    if (!X || !Y || !p0) return fail(LM_EINVAL, "NULL buffer");
    if (!(o->h > 0.0) || !is_finite(o->h)) return fail(LM_EINVAL, "h must be positive");
    if (!(o->tol > 0.0) || !is_finite(o->tol)) return fail(LM_EINVAL, "tol must be positive");
    if (o->max_iter < 0) return fail(LM_EINVAL, "max_iter must be >= 0");
    if (o->steps < 1) return fail(LM_EINVAL, "steps must be >= 1");
    if (o->stop_rule != 0 && o->stop_rule != 1) return fail(LM_EINVAL, "stop_rule must be 0 or 1");
    if (o->cg_max_iter < 0 || !(o->cg_rtol >= 0.0)) return fail(LM_EINVAL, "bad CG settings");
    if (o->hist_len < 0 || (o->hist_len > 0 && !o->resid_hist)) return fail(LM_EINVAL, "bad history buffer");
    if (o->solver < LM_SOLVE_AUTO || o->solver > LM_SOLVE_DENSE) return fail(LM_EINVAL, "unknown solver %d", o->solver);
    if (!(o->f32_switch >= 0.0) || !is_finite(o->f32_switch)) return fail(LM_EINVAL, "f32_switch must be >= 0");
    return LM_OK;
}

// Device buffers of one feedback match.
struct FeedbackWork {
    double *qd = nullptr, *pd = nullptr, *e = nullptr, *delta = nullptr, *part = nullptr, *red = nullptr,
           *rdev = nullptr;
    double *aq = nullptr, *ap = nullptr, *bq = nullptr, *bp = nullptr, *cq = nullptr, *cp = nullptr;
    float *qf = nullptr, *pf = nullptr, *aqf = nullptr, *apf = nullptr, *bqf = nullptr, *bpf = nullptr,
          *cqf = nullptr, *cpf = nullptr;
    double* q1 = nullptr;     // q(1) in the caller's order (== qd unless the shoot is reordered)
    bool dense = false;       // K-solves with the dense factor (else CG)
    DenseFactor fac;
    bool ordered = false;     // cutoff mode: shoots run in the Morton order of X
    Ordering ord;
    CgBuffers cg;

    lm_status alloc(Workspace& ws, const lm_params* prm, int64_t n, const double* X, hipStream_t st)
    {
        const int64_t m = (int64_t)prm->dim * n;
        ordered = prm->cutoff > 0.0;
        if (ordered) {
            if (n > kMaxCutN) return fail(LM_EINVAL, "cutoff mode needs n < 2^31");
            LM_TRY(ord.alloc(ws, n));
            LM_TRY(ord.compute<double>(prm->dim, X, n, ws, st));
            LM_TRY(ws.get(&q1, m));
        }
        LM_TRY(ws.get(&qd, m));
        LM_TRY(ws.get(&pd, m));
        LM_TRY(ws.get(&e, m));
        LM_TRY(ws.get(&delta, m));
        LM_TRY(ws.get(&part, part_elems(prm, n, n)));
        LM_TRY(ws.get(&red, lm::reduce_blocks(m)));
        LM_TRY(ws.get(&rdev, 1));
        if (prm->dtype == LM_F32) {
            LM_TRY(ws.get(&qf, m));
            LM_TRY(ws.get(&pf, m));
            LM_TRY(ws.get(&aqf, m));
            LM_TRY(ws.get(&apf, m));
            LM_TRY(ws.get(&bqf, m));
            LM_TRY(ws.get(&bpf, m));
            LM_TRY(ws.get(&cqf, m));
            LM_TRY(ws.get(&cpf, m));
        }
        // double-precision stage buffers (single-precision matches may switch to them)
        LM_TRY(ws.get(&aq, m));
        LM_TRY(ws.get(&ap, m));
        LM_TRY(ws.get(&bq, m));
        LM_TRY(ws.get(&bp, m));
        LM_TRY(ws.get(&cq, m));
        LM_TRY(ws.get(&cp, m));
        if (!ordered) q1 = qd;
        return cg_alloc(ws, prm, n, &cg);
    }

    // Factor K(X) once when the dense solver is chosen.
    lm_status prepare_solver(Workspace& ws, const lm_params* prm, const lm_match_opts* o, int64_t n,
                             const double* X, hipStream_t st)
    {
        LM_TRY(pick_solver(o->solver, n, &dense));
        // a match with single-precision shoots steers by solves that need not be exact: its
        // factor's trailing updates multiply in single precision
        if (dense) LM_TRY(dense_factor(prm, n, X, ws, &fac, st, prm->dtype == LM_F32));
        return LM_OK;
    }
};

// Algorithm 1, steps 1-2: q(1) of the shoot from (X, p) into w.q1, and r = max |Y - q(1)|
// (read back to the host: it decides the next launch).
// still: p is zero, so no landmark moves and q(1) = X (the double-precision RK4 steps give
// exactly that: every increment is a sum of products with a zero momentum); the shoot is then
// not integrated.
lm_status feedback_shoot_residual(const lm_params* prm, const lm_match_opts* o, int64_t n, const double* X,
                                  const double* Y, const double* p, FeedbackWork& w, double* r, hipStream_t st,
                                  hipEvent_t after_shoot = nullptr, bool still = false)
{
    const int dim = prm->dim;
    const int64_t m = (int64_t)dim * n;
    const int64_t* perm = w.ord.perm;
    double* box = w.ordered ? w.ord.box : nullptr;
    if (still) {
        LM_HIP(hipMemcpyAsync(w.q1, X, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else if (prm->dtype == LM_F32) {
        // single-precision shoot; the momenta, the residual and the solve stay in double
        if (w.ordered) {
            LM_HIP((lm::launch_permute<float, double>(w.qf, X, perm, n, dim, false, st)));
            LM_HIP((lm::launch_permute<float, double>(w.pf, p, perm, n, dim, false, st)));
        } else {
            LM_HIP((lm::launch_convert<float, double>(w.qf, X, m, st)));
            LM_HIP((lm::launch_convert<float, double>(w.pf, p, m, st)));
        }
        LM_TRY(shoot_inplace<float>(prm, n, w.qf, w.pf, 1.0, o->steps, w.aqf, w.apf, w.bqf, w.bpf, w.cqf, w.cpf,
                                    w.part, st, box));
        if (w.ordered)
            LM_HIP((lm::launch_permute<double, float>(w.q1, w.qf, perm, n, dim, true, st)));
        else
            LM_HIP((lm::launch_convert<double, float>(w.qd, w.qf, m, st)));
    } else {
        if (w.ordered) {
            LM_HIP((lm::launch_permute<double, double>(w.qd, X, perm, n, dim, false, st)));
            LM_HIP((lm::launch_permute<double, double>(w.pd, p, perm, n, dim, false, st)));
        } else {
            LM_HIP(hipMemcpyAsync(w.qd, X, m * sizeof(double), hipMemcpyDeviceToDevice, st));
            LM_HIP(hipMemcpyAsync(w.pd, p, m * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
        LM_TRY(shoot_inplace<double>(prm, n, w.qd, w.pd, 1.0, o->steps, w.aq, w.ap, w.bq, w.bp, w.cq, w.cp, w.part,
                                     st, box));
        if (w.ordered) LM_HIP((lm::launch_permute<double, double>(w.q1, w.qd, perm, n, dim, true, st)));
    }
    if (after_shoot) LM_HIP(hipEventRecord(after_shoot, st));
    LM_HIP((lm::launch_maxabsdiff<double, double>(Y, w.q1, m, w.red, w.rdev, st)));
    LM_HIP(hipMemcpyAsync(r, w.rdev, sizeof(double), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

// Algorithm 1, steps 3-4 with M = h I: u <- u + h e, i.e. p <- p + h (K(X) + tau I)^{-1} e,
// e = Y - q(1) taken from w.qd.
lm_status feedback_update(const lm_params* prm, const lm_match_opts* o, int64_t n, const double* X, const double* Y,
                          double* p, FeedbackWork& w, int32_t* cg_iters, hipStream_t st)
{
    const int64_t m = (int64_t)prm->dim * n;
    const double cg_rtol = o->cg_rtol > 0.0 ? o->cg_rtol : 1e-13;
    const int64_t cgdef = 20 * n + 100 < 10000 ? 20 * n + 100 : 10000;
    const int32_t cg_max = o->cg_max_iter > 0 ? o->cg_max_iter : (int32_t)cgdef;
    LM_HIP(lm::launch_sub(w.e, Y, w.q1, m, st));
    if (w.dense) {
        *cg_iters = 0;
        LM_TRY(dense_solve(w.fac, prm->dim, w.e, w.delta, st));
    } else {
        LM_TRY(ksolve_impl(prm, n, X, w.e, w.delta, cg_rtol, cg_max, cg_iters, w.cg, w.part, st));
    }
    LM_HIP(lm::launch_axpy(p, p, o->h, w.delta, m, st));
    return LM_OK;
}

// ---- Reverse mode ------------------------------------------------------------------------

// One VJP launch: J(q, p)^T (a, b) handled by the epilogue e.
lm_status vjp_eval(const lm_params* prm, int64_t n, const double* q, const double* p, const double* a,
                   const double* b, const lm::AdjEpi& e, double* part, hipStream_t st)
{
    lm::PairPlan pl = lm::plan_pair(n, n, false, true, lm::SYM_VJP);
    lm::VjpArgs A{};
    A.q = q;
    A.p = p;
    A.a = a;
    A.b = b;
    A.n = n;
    A.jchunk = pl.jchunk;
    const double sg = prm->sigma;
    if (prm->kernel == LM_KERNEL_CONON) {
        A.kq = -lmh::kLog2e / sg;
        A.c1 = 1.0 / sg;
        A.c2 = 0.0;
    } else {
        A.kq = -lmh::kLog2e / (sg * sg);
        A.c1 = 2.0 / (sg * sg);
        A.c2 = -4.0 / (sg * sg * sg * sg);
    }
    A.pack = part;
    A.part = part + 4 * (int64_t)prm->dim * n;
    A.epi = e;
    LM_HIP(lm::launch_vjp(prm->dim, prm->kernel, A, pl, st));
    return LM_OK;
}

// Buffers of a checkpointed adjoint: the states at segment starts, the stage inputs of one
// segment (slot(i, s) = stage s+1 input of step i of the segment, slot(i+1, 0) its output),
// the RK4 running sum, two cotangent and two lambda buffers.  A state is (q, p) = 2 dim n.
struct AdjointWork {
    int64_t m = 0;            // dim * n
    int32_t steps = 0, ckpt = 0, nseg = 0;
    double dt = 0.0;
    double *ckpts = nullptr, *slots = nullptr, *acc = nullptr, *part = nullptr;
    double *L0 = nullptr, *L1 = nullptr, *C0 = nullptr, *C1 = nullptr;

    double* slot(int32_t i, int s) const { return slots + ((int64_t)i * 4 + s) * 2 * m; }
    double* ck(int32_t seg) const { return ckpts + (int64_t)seg * 2 * m; }
    int32_t seg_steps(int32_t seg) const { return (seg + 1) * ckpt <= steps ? ckpt : steps - seg * ckpt; }

    lm_status alloc(Workspace& ws, const lm_params* prm, int64_t n, double t1, int32_t nsteps, int32_t every)
    {
        m = (int64_t)prm->dim * n;
        steps = nsteps;
        ckpt = (every <= 0 || every > nsteps) ? nsteps : every;
        nseg = (steps + ckpt - 1) / ckpt;
        dt = t1 / steps;
        LM_TRY(ws.get(&ckpts, (int64_t)nseg * 2 * m));
        LM_TRY(ws.get(&slots, ((int64_t)ckpt * 4 + 1) * 2 * m));
        LM_TRY(ws.get(&acc, 2 * m));
        LM_TRY(ws.get(&part, vjp_part_elems(prm, n)));
        LM_TRY(ws.get(&L0, 2 * m));
        LM_TRY(ws.get(&L1, 2 * m));
        LM_TRY(ws.get(&C0, 2 * m));
        LM_TRY(ws.get(&C1, 2 * m));
        return LM_OK;
    }
};

// One RK4 step of the segment: stage inputs into slot(i, 1..3), the step output into
// slot(i + 1, 0).
lm_status rk_step_slots(const lm_params* prm, int64_t n, const AdjointWork& W, int32_t i, hipStream_t st)
{
    const int64_t m = W.m;
    lm::EpiArgs<double> e{};
    e.dt = W.dt;
    e.tau = prm->tau;
    double* y = W.slot(i, 0);
    e.base_q = y;
    e.base_p = y + m;
    e.acc_q = W.acc;
    e.acc_p = W.acc + m;
    for (int k = 0; k < 4; ++k) {
        const double* in = W.slot(i, k);
        double* out = (k < 3) ? W.slot(i, k + 1) : W.slot(i + 1, 0);
        e.kind = lm::EPI_RK1 + k;
        e.in_p = in + m;
        e.out_q = out;
        e.out_p = out + m;
        LM_TRY(pair_eval<double>(prm, true, in, in + m, n, in, in + m, n, e, W.part, st));
    }
    return LM_OK;
}

// Forward pass keeping a state every `ckpt` steps; the slots end up holding the last
// segment, whose final output is the state at t1.  Returns that state's pointer.
lm_status adjoint_forward(const lm_params* prm, int64_t n, const double* q0, const double* p0, AdjointWork& W,
                          const double** final_state, hipStream_t st)
{
    const int64_t m = W.m;
    LM_HIP(hipMemcpyAsync(W.ck(0), q0, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(hipMemcpyAsync(W.ck(0) + m, p0, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int32_t seg = 0; seg < W.nseg; ++seg) {
        const int32_t ns = W.seg_steps(seg);
        LM_HIP(hipMemcpyAsync(W.slot(0, 0), W.ck(seg), 2 * m * sizeof(double), hipMemcpyDeviceToDevice, st));
        for (int32_t i = 0; i < ns; ++i) LM_TRY(rk_step_slots(prm, n, W, i, st));
        if (seg + 1 < W.nseg)
            LM_HIP(hipMemcpyAsync(W.ck(seg + 1), W.slot(ns, 0), 2 * m * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    *final_state = W.slot(W.seg_steps(W.nseg - 1), 0);
    return LM_OK;
}

// Reverse sweep from the cotangent in W.L0 (of the state at t1) to that of the initial
// state, returned through *lam.  Expects the slots to hold the last segment.
lm_status adjoint_reverse(const lm_params* prm, int64_t n, AdjointWork& W, const double** lam, hipStream_t st)
{
    const int64_t m = W.m;
    const double dt = W.dt;
    double *Lin = W.L0, *Lout = W.L1;
    for (int32_t seg = W.nseg - 1; seg >= 0; --seg) {
        const int32_t ns = W.seg_steps(seg);
        if (seg < W.nseg - 1) {   // recompute the segment's stage inputs from its checkpoint
            LM_HIP(hipMemcpyAsync(W.slot(0, 0), W.ck(seg), 2 * m * sizeof(double), hipMemcpyDeviceToDevice, st));
            for (int32_t i = 0; i < ns; ++i) LM_TRY(rk_step_slots(prm, n, W, i, st));
        }
        for (int32_t i = ns - 1; i >= 0; --i) {
            lm::AdjEpi e{};
            e.tau = prm->tau;
            e.abar_q = Lin;
            e.abar_p = Lin + m;
            e.lam_q = Lout;
            e.lam_p = Lout + m;
            // stage 4: cotangent dt/6 abar, next = dt/3 abar + dt Yb4
            const double* Y = W.slot(i, 3);
            e.kind = lm::ADJ_FIRST;
            e.cscale = dt / 6.0;
            e.ca = dt / 3.0;
            e.cy = dt;
            e.cot_q = Lin;
            e.nxt_q = W.C0;
            e.nxt_p = W.C0 + m;
            LM_TRY(vjp_eval(prm, n, Y, Y + m, Lin, Lin + m, e, W.part, st));
            // stage 3: next = dt/3 abar + dt/2 Yb3
            Y = W.slot(i, 2);
            e.kind = lm::ADJ_MID;
            e.cscale = 1.0;
            e.ca = dt / 3.0;
            e.cy = 0.5 * dt;
            e.cot_q = W.C0;
            e.nxt_q = W.C1;
            e.nxt_p = W.C1 + m;
            LM_TRY(vjp_eval(prm, n, Y, Y + m, W.C0, W.C0 + m, e, W.part, st));
            // stage 2: next = dt/6 abar + dt/2 Yb2
            Y = W.slot(i, 1);
            e.ca = dt / 6.0;
            e.cy = 0.5 * dt;
            e.cot_q = W.C1;
            e.nxt_q = W.C0;
            e.nxt_p = W.C0 + m;
            LM_TRY(vjp_eval(prm, n, Y, Y + m, W.C1, W.C1 + m, e, W.part, st));
            // stage 1
            Y = W.slot(i, 0);
            e.kind = lm::ADJ_LAST;
            e.cot_q = W.C0;
            e.nxt_q = e.nxt_p = nullptr;
            LM_TRY(vjp_eval(prm, n, Y, Y + m, W.C0, W.C0 + m, e, W.part, st));
            std::swap(Lin, Lout);
        }
    }
    *lam = Lin;
    return LM_OK;
}


lm_status check_adjoint_params(const lm_params* prm)
{
    LM_TRY(check_params(prm));
    if (prm->dtype != LM_F64) return fail(LM_EUNSUPPORTED, "the adjoint is provided in double precision only");
    if (prm->cutoff > 0.0) return fail(LM_EUNSUPPORTED, "the adjoint is provided for every-pair sums only (cutoff = 0)");
    return LM_OK;
}

// Buffers of energy/gradient evaluations: the adjoint's, plus K p0, the residual reductions
// and q(1).
struct EnergyWork {
    AdjointWork W;
    double *v = nullptr, *red = nullptr, *dots = nullptr, *red2 = nullptr, *rmax = nullptr;
    int64_t m = 0;
    lm_status alloc(Workspace& ws, const lm_params* prm, int64_t n, int32_t steps, int32_t ckpt_every)
    {
        LM_TRY(W.alloc(ws, prm, n, 1.0, steps, ckpt_every));
        m = W.m;
        LM_TRY(ws.get(&v, m));
        LM_TRY(ws.get(&red, (int64_t)lm::reduce_blocks(m) * 3));
        LM_TRY(ws.get(&dots, 8));
        LM_TRY(ws.get(&red2, lm::reduce_blocks(m)));
        LM_TRY(ws.get(&rmax, 1));
        return LM_OK;
    }
};

// E(p0) = reg/2 p0^T K(X) p0 + lam/2 |q(1) - Y|^2 and grad = reg K(X) p0 + J^T (lam (q(1) - Y), 0);
// *resid (nullable) receives max |q(1) - Y|.
lm_status energy_grad_impl(const lm_params* prm, int64_t n, const double* X, const double* Y, const double* p0,
                           double lam, double reg, EnergyWork& E, double* E_out, double* grad, double* q1,
                           double* resid, hipStream_t st)
{
    const int dim = prm->dim;
    AdjointWork& W = E.W;
    const int64_t m = W.m;
    lm::EpiArgs<double> ev{};
    ev.kind = lm::EPI_STORE;
    ev.tau = 0.0;
    ev.out_q = E.v;
    LM_TRY(pair_eval<double>(prm, false, X, p0, n, X, p0, n, ev, W.part, st));
    LM_HIP(lm::launch_dots(p0, E.v, n, dim, E.red, E.dots, st));
    const double* yT = nullptr;
    LM_TRY(adjoint_forward(prm, n, X, p0, W, &yT, st));
    if (q1) LM_HIP(hipMemcpyAsync(q1, yT, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(lm::launch_sub(W.C0, yT, Y, m, st));
    LM_HIP(lm::launch_dots(W.C0, W.C0, n, dim, E.red, E.dots + 3, st));
    if (resid) LM_HIP((lm::launch_maxabsdiff<double, double>(yT, Y, m, E.red2, E.rmax, st)));
    LM_HIP(lm::launch_scale(W.L0, lam, W.C0, m, st));
    LM_HIP(lm::launch_zero(W.L0 + m, m, st));
    const double* lamv = nullptr;
    LM_TRY(adjoint_reverse(prm, n, W, &lamv, st));
    LM_HIP(lm::launch_axpy(grad, lamv + m, reg, E.v, m, st));
    double hd[7] = {0, 0, 0, 0, 0, 0, 0};
    LM_HIP(hipMemcpyAsync(hd, E.dots, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (resid) LM_HIP(hipMemcpyAsync(hd + 6, E.rmax, sizeof(double), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    double e1 = 0.0, e2 = 0.0;
    for (int c = 0; c < dim; ++c) {
        e1 += hd[c];
        e2 += hd[3 + c];
    }
    *E_out = 0.5 * reg * e1 + 0.5 * lam * e2;
    if (resid) *resid = hd[6];
    return LM_OK;
}

// Full dot product of two m-vectors (read back to the host).
lm_status dot_host(const double* x, const double* y, int64_t m, EnergyWork& E, double* out, hipStream_t st)
{
    LM_HIP(lm::launch_dots(x, y, m, 1, E.red, E.dots + 6, st));
    LM_HIP(hipMemcpyAsync(out, E.dots + 6, sizeof(double), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

lm_status maxabs_host(const double* x, int64_t m, const double* zeros, EnergyWork& E, double* out, hipStream_t st)
{
    LM_HIP((lm::launch_maxabsdiff<double, double>(x, zeros, m, E.red2, E.rmax, st)));
    LM_HIP(hipMemcpyAsync(out, E.rmax, sizeof(double), hipMemcpyDeviceToHost, st));
    LM_HIP(hipStreamSynchronize(st));
    return LM_OK;
}

// Limited-memory BFGS (two-loop recursion) with a backtracking Armijo line search that also
// expands a first step of unit length in p.  Every vector operation runs on the GPU; the
// host keeps the scalars (dot products, step lengths) that decide the next launch.
lm_status lbfgs_impl(const lm_params* prm, const lm_lbfgs_opts* o, int64_t n, const double* X, const double* Y,
                     double* x, lm_lbfgs_info* info, EnergyWork& E, Workspace& ws, hipStream_t st)
{
    const int64_t m = (int64_t)prm->dim * n;
    const int hm = o->history > 0 ? o->history : 8;
    double *g, *d, *xn, *gn, *xt, *gt, *qv, *zeros, *S, *Yh;
    LM_TRY(ws.get(&xt, m));
    LM_TRY(ws.get(&gt, m));
    LM_TRY(ws.get(&g, m));
    LM_TRY(ws.get(&d, m));
    LM_TRY(ws.get(&xn, m));
    LM_TRY(ws.get(&gn, m));
    LM_TRY(ws.get(&qv, m));
    LM_TRY(ws.get(&zeros, m));
    LM_TRY(ws.get(&S, (int64_t)hm * m));
    LM_TRY(ws.get(&Yh, (int64_t)hm * m));
    LM_HIP(lm::launch_zero(zeros, m, st));
    std::vector<double> rho(hm, 0.0), alpha(hm, 0.0);
    int stored = 0, newest = -1;
    double f = 0.0, resid = 0.0;
    LM_TRY(energy_grad_impl(prm, n, X, Y, x, o->lam, o->reg, E, &f, g, nullptr, &resid, st));
    info->evals = 1;
    double g0 = 0.0;
    LM_TRY(maxabs_host(g, m, zeros, E, &g0, st));
    double gmax = g0;
    lm_status result = LM_ENOTCONV;
    int it = 0;
    for (it = 0;; ++it) {
        if (!is_finite(f) || !is_finite(gmax)) {
            result = fail(LM_EDIVERGED, "L-BFGS: non-finite energy or gradient");
            break;
        }
        if (gmax <= o->gtol * g0 || (o->match_tol > 0.0 && resid < o->match_tol)) {
            result = LM_OK;
            break;
        }
        if (it >= o->max_iter) {
            result = fail(LM_ENOTCONV, "L-BFGS: %d iterations (max|grad| %.3g, residual %.3g)", it, gmax, resid);
            break;
        }
        // two-loop recursion: d = -H g
        LM_HIP(hipMemcpyAsync(qv, g, m * sizeof(double), hipMemcpyDeviceToDevice, st));
        for (int k = 0; k < stored; ++k) {
            const int i = (newest - k + hm) % hm;
            double sq = 0.0;
            LM_TRY(dot_host(S + (int64_t)i * m, qv, m, E, &sq, st));
            alpha[i] = rho[i] * sq;
            LM_HIP(lm::launch_axpy(qv, qv, -alpha[i], Yh + (int64_t)i * m, m, st));
        }
        double gamma;
        if (stored > 0) {
            double sy = 0.0, yy = 0.0;
            LM_TRY(dot_host(S + (int64_t)newest * m, Yh + (int64_t)newest * m, m, E, &sy, st));
            LM_TRY(dot_host(Yh + (int64_t)newest * m, Yh + (int64_t)newest * m, m, E, &yy, st));
            gamma = sy / yy;
        } else {
            double gg = 0.0;
            LM_TRY(dot_host(g, g, m, E, &gg, st));
            gamma = 1.0 / std::sqrt(gg);       // first step: unit length in p
        }
        LM_HIP(lm::launch_scale(qv, gamma, qv, m, st));
        for (int k = stored - 1; k >= 0; --k) {
            const int i = (newest - k + hm) % hm;
            double yr = 0.0;
            LM_TRY(dot_host(Yh + (int64_t)i * m, qv, m, E, &yr, st));
            const double beta = rho[i] * yr;
            LM_HIP(lm::launch_axpy(qv, qv, alpha[i] - beta, S + (int64_t)i * m, m, st));
        }
        LM_HIP(lm::launch_scale(d, -1.0, qv, m, st));
        double gd = 0.0;
        LM_TRY(dot_host(g, d, m, E, &gd, st));
        if (!(gd < 0.0)) {   // not a descent direction: restart from the scaled gradient
            stored = 0;
            double gg = 0.0;
            LM_TRY(dot_host(g, g, m, E, &gg, st));
            LM_HIP(lm::launch_scale(d, -1.0 / std::sqrt(gg), g, m, st));
            gd = -std::sqrt(gg);
        }
        // backtracking Armijo (c1 = 1e-4); on the first iteration also expand while it pays
        double t = 1.0, fn = 0.0, rn = 0.0;
        bool ok = false;
        for (int ls = 0; ls < 40; ++ls) {
            LM_HIP(lm::launch_axpy(xn, x, t, d, m, st));
            LM_TRY(energy_grad_impl(prm, n, X, Y, xn, o->lam, o->reg, E, &fn, gn, nullptr, &rn, st));
            ++info->evals;
            if (is_finite(fn) && fn <= f + 1e-4 * t * gd) {
                ok = true;
                break;
            }
            t *= 0.5;
        }
        if (!ok) {
            result = fail(LM_ENOTCONV, "L-BFGS: line search failed at iteration %d", it);
            break;
        }
        if (it == 0) {
            // expansion of the very first step: double t while the energy keeps falling
            for (int ex = 0; ex < 30; ++ex) {
                double f2 = 0.0, r2 = 0.0;
                LM_HIP(lm::launch_axpy(xt, x, 2.0 * t, d, m, st));
                LM_TRY(energy_grad_impl(prm, n, X, Y, xt, o->lam, o->reg, E, &f2, gt, nullptr, &r2, st));
                ++info->evals;
                if (!(is_finite(f2) && f2 < fn)) break;
                t *= 2.0;
                fn = f2;
                rn = r2;
                std::swap(xn, xt);
                std::swap(gn, gt);
            }
        }
        // history pair s = xn - x, y = gn - g
        const int slot = (newest + 1) % hm;
        double* sv = S + (int64_t)slot * m;
        double* yv = Yh + (int64_t)slot * m;
        LM_HIP(lm::launch_sub(sv, xn, x, m, st));
        LM_HIP(lm::launch_sub(yv, gn, g, m, st));
        double sy = 0.0;
        LM_TRY(dot_host(sv, yv, m, E, &sy, st));
        if (sy > 0.0) {
            rho[slot] = 1.0 / sy;
            newest = slot;
            if (stored < hm) ++stored;
        }
        LM_HIP(hipMemcpyAsync(x, xn, m * sizeof(double), hipMemcpyDeviceToDevice, st));
        LM_HIP(hipMemcpyAsync(g, gn, m * sizeof(double), hipMemcpyDeviceToDevice, st));
        f = fn;
        resid = rn;
        LM_TRY(maxabs_host(g, m, zeros, E, &gmax, st));
    }
    info->iters = it;
    info->E = f;
    info->gnorm_inf = gmax;
    info->resid_inf = resid;
    return result;
}

// ---------------------------------------------------------------------------------------
// lm_shoot_noalloc: lm_shoot with its scratch memory (stage buffers, RK4 running sums and
// the pair kernels' partial sums) carved out of one fixed device array instead of the
// stream-ordered allocator, for callers that cannot allocate.
// ---------------------------------------------------------------------------------------

// The fixed scratch array: one copy per GPU, resident from the library's first use on that
// GPU until the process ends.  Host code never uses this name as an address (on the host it
// is a stand-in, not device memory); scratch_base() gives each device's own copy's address.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_base[kMaxDevices] = {};

// Device address of device `dev`'s copy of the scratch array; `dev` must be the current
// device.  Looked up once per device (hipGetSymbolAddress) and kept.
lm_status scratch_base(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LM_EINVAL, "device %d is beyond the %d tracked", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_base[dev]) {
        void* ptr = nullptr;
        LM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LM_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch_base[dev] = (unsigned char*)ptr;
    }
    *out = g_scratch_base[dev];
    return LM_OK;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch bytes of a shoot of n points: six state arrays (two stage buffers and the RK4
// running sum, for q and p) and the partial sums of any pair kernel the plan may pick.
size_t noalloc_bytes(const lm_params* prm, int64_t n)
{
    const size_t es = prm->dtype == LM_F64 ? sizeof(double) : sizeof(float);
    return 6 * align256((size_t)prm->dim * (size_t)n * es) + align256((size_t)part_elems(prm, n, n) * sizeof(double));
}

template <class T>
lm_status shoot_noalloc_t(const lm_params* prm, int64_t n, const T* q0, const T* p0, double t1, int32_t steps,
                          T* q1, T* p1, unsigned char* base, hipStream_t st)
{
    const size_t sb = align256((size_t)prm->dim * (size_t)n * sizeof(T));
    T* buf[6];
    for (int k = 0; k < 6; ++k) buf[k] = (T*)(base + k * sb);
    double* part = (double*)(base + 6 * sb);
    const int64_t m = (int64_t)prm->dim * n;
    if (q1 != q0) LM_HIP(hipMemcpyAsync(q1, q0, m * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (p1 != p0) LM_HIP(hipMemcpyAsync(p1, p0, m * sizeof(T), hipMemcpyDeviceToDevice, st));
    return shoot_inplace<T>(prm, n, q1, p1, t1, steps, buf[0], buf[1], buf[2], buf[3], buf[4], buf[5], part, st);
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================

extern "C" {

const char* lm_last_error(void) { return lmh::last_error(); }

const char* lm_version(void) { return "liblm 0.1 (gfx950)"; }

lm_status lm_rhs(const lm_params* prm, int64_t n, const void* q, const void* p, void* dq, void* dp, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!q || !p || !dq || !dp) return fail(LM_EINVAL, "NULL buffer");
    if (dq == q || dq == p || dp == q || dp == p) return fail(LM_EINVAL, "dq/dp must not alias q/p");
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F64)
        return rhs_t<double>(prm, n, (const double*)q, (const double*)p, (double*)dq, (double*)dp, st);
    return rhs_t<float>(prm, n, (const float*)q, (const float*)p, (float*)dq, (float*)dp, st);
}

lm_status lm_pair_plan(const lm_params* prm, int64_t n, lm_plan_info* info)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!info) return fail(LM_EINVAL, "NULL info");
    const bool cut = prm->cutoff > 0.0;
    const lm::PairPlan pl = lm::plan_pair(n, n, cut, true, prm->dtype == LM_F32 ? lm::SYM_F32 : lm::SYM_F64);
    info->symmetric = pl.sym_waves > 0;
    info->waves = pl.sym_waves > 0 ? pl.sym_waves : lm::kWaves;
    info->workgroups = pl.sym_waves > 0 ? pl.sym_nsb * (pl.sym_nsb + 1) / 2 : pl.itiles * pl.nsplit;
    info->partial_slots = pl.nsplit;
    info->small = !cut && lm::small_path(n, prm->dim, prm->dtype == LM_F32);
    info->rows = pl.sym_waves > 0 ? pl.sym_rows : 1;
    return LM_OK;
}

lm_status lm_shoot(const lm_params* prm, int64_t n, const void* q0, const void* p0, double t1, int32_t steps,
                   void* q1, void* p1, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!q0 || !p0 || !q1 || !p1) return fail(LM_EINVAL, "NULL buffer");
    if (steps < 1) return fail(LM_EINVAL, "steps must be >= 1 (got %d)", steps);
    if (!is_finite(t1)) return fail(LM_EINVAL, "t1 must be finite");
    if (q1 == p1) return fail(LM_EINVAL, "q1 and p1 must be distinct buffers");
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F64)
        return shoot_t<double>(prm, n, (const double*)q0, (const double*)p0, t1, steps, (double*)q1, (double*)p1,
                               st);
    return shoot_t<float>(prm, n, (const float*)q0, (const float*)p0, t1, steps, (float*)q1, (float*)p1, st);
}

lm_status lm_hamiltonian(const lm_params* prm, int64_t n, const void* q, const void* p, double* H_out,
                         void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!q || !p || !H_out) return fail(LM_EINVAL, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F64) return hamiltonian_f64(prm, n, (const double*)q, (const double*)p, H_out, st);
    const int64_t m = (int64_t)prm->dim * n;
    Workspace ws(st);
    double *qd, *pd;
    LM_TRY(ws.get(&qd, m));
    LM_TRY(ws.get(&pd, m));
    LM_HIP((lm::launch_convert<double, float>(qd, (const float*)q, m, st)));
    LM_HIP((lm::launch_convert<double, float>(pd, (const float*)p, m, st)));
    return hamiltonian_f64(prm, n, qd, pd, H_out, st);
}

lm_status lm_ksolve(const lm_params* prm, int64_t n, const double* X, const double* b, double* x, double rtol,
                    int32_t max_iter, int32_t solver, int32_t* iters_out, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!X || !b || !x) return fail(LM_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    bool dense = false;
    LM_TRY(pick_solver(solver, n, &dense));
    Workspace ws(st);
    if (iters_out) *iters_out = 0;
    if (dense) {
        DenseFactor f;
        LM_TRY(dense_factor(prm, n, X, ws, &f, st));
        LM_TRY(dense_solve(f, prm->dim, b, x, st));
        LM_HIP(hipStreamSynchronize(st));
        return LM_OK;
    }
    if (!(rtol > 0.0) || !is_finite(rtol)) return fail(LM_EINVAL, "rtol must be positive");
    if (max_iter < 1) return fail(LM_EINVAL, "max_iter must be >= 1");
    CgBuffers cg;
    double* part;
    LM_TRY(cg_alloc(ws, prm, n, &cg));
    LM_TRY(ws.get(&part, part_elems(prm, n, n)));
    return ksolve_impl(prm, n, X, b, x, rtol, max_iter, iters_out, cg, part, st);
}

lm_status lm_feedback_match(const lm_params* prm, const lm_match_opts* o, int64_t n, const double* X,
                            const double* Y, double* p0, double* q1_out, lm_match_info* info, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!info) return fail(LM_EINVAL, "info is NULL");
    LM_TRY(check_match_args(o, X, Y, p0));
    hipStream_t st = (hipStream_t)stream;
    std::memset(info, 0, sizeof *info);
    Workspace ws(st);
    FeedbackWork w;
    LM_TRY(w.alloc(ws, prm, n, X, st));
    EventTimer timer;
    LM_TRY(timer.init());
    LM_HIP(hipEventRecord(timer.ev[0], st));
    LM_TRY(w.prepare_solver(ws, prm, o, n, X, st));
    LM_HIP(hipEventRecord(timer.ev[1], st));
    LM_HIP(hipEventSynchronize(timer.ev[1]));
    if (w.dense) info->factor_ms = timer.ms(0, 1);

    lm_status result = LM_OK;
    double r = 0.0, prev_step = INFINITY, prev_r = INFINITY;
    int32_t k = 0;   // momentum updates made
    // single-precision shoots until the residual drops below f32_switch (if set), then double
    lm_params p64 = *prm;
    p64.dtype = LM_F64;
    const bool may_switch = prm->dtype == LM_F32 && o->f32_switch > 0.0;
    bool fp64 = prm->dtype == LM_F64;
    // zero initial momenta (the paper's starting guess): the first shoot is the identity map
    bool still = false;
    {
        const int64_t m = (int64_t)prm->dim * n;
        double pmax = 1.0;
        LM_HIP(lm::launch_zero(w.delta, m, st));
        LM_HIP((lm::launch_maxabsdiff<double, double>(p0, w.delta, m, w.red, w.rdev, st)));
        LM_HIP(hipMemcpyAsync(&pmax, w.rdev, sizeof(double), hipMemcpyDeviceToHost, st));
        LM_HIP(hipStreamSynchronize(st));
        still = pmax == 0.0;

    }
    for (int32_t shot = 0;; ++shot) {
        // Algorithm 1, steps 1-2: shoot (X, p) to t = 1, residual r = max |Y - q(1)|
        LM_HIP(hipEventRecord(timer.ev[0], st));
        LM_TRY(feedback_shoot_residual(fp64 ? &p64 : prm, o, n, X, Y, p0, w, &r, st, timer.ev[1],
                                       shot == 0 && still));
        info->shoot_ms += timer.ms(0, 1);
        if (!(shot == 0 && still)) ++info->shoots;
        if (shot < o->hist_len) o->resid_hist[shot] = r;
        if (!is_finite(r)) {
            result = fail(LM_EDIVERGED, "feedback iteration %d: non-finite residual", k);
            break;
        }
        bool hold = false;   // re-shoot the same momenta in double precision
        if (may_switch && !fp64) {
            if (r < o->f32_switch) fp64 = true;
            if (r < o->tol || r >= lm::kF32Stall * prev_r) {
                // below tol, or at the single-precision floor (the residual stopped falling)
                hold = true;
                fp64 = true;
            }
        }
        prev_r = r;
        if (!hold && (o->stop_rule == 0 ? (r < o->tol) : (k >= 1 && prev_step < o->tol))) break;
        if (k >= o->max_iter) {
            result = fail(LM_ENOTCONV, "feedback: %d updates without reaching tol %.3g (residual %.3g)", k, o->tol, r);
            break;
        }
        if (hold) continue;
        // steps 3-4: u <- u + h e, i.e. p <- p + h (K + tau I)^{-1} e
        int32_t cgit = 0;
        LM_HIP(hipEventRecord(timer.ev[2], st));
        lm_status s = feedback_update(prm, o, n, X, Y, p0, w, &cgit, st);
        info->cg_iters += cgit;
        if (s != LM_OK) {
            result = s;
            break;
        }
        LM_HIP(hipEventRecord(timer.ev[3], st));
        LM_HIP(hipEventSynchronize(timer.ev[3]));
        info->solve_ms += timer.ms(2, 3);
        prev_step = o->h * r;
        ++k;
    }
    info->iters = k;
    info->resid_inf = r;
    if (q1_out) LM_HIP(hipMemcpyAsync(q1_out, w.q1, (int64_t)prm->dim * n * sizeof(double), hipMemcpyDeviceToDevice, st));
    double H = NAN;
    lm_status hs = hamiltonian_f64(prm, n, X, p0, &H, st);
    info->H = H;
    if (result == LM_OK && hs != LM_OK) return hs;
    return result;
}

lm_status lm_feedback_step(const lm_params* prm, const lm_match_opts* o, int64_t n, const double* X,
                           const double* Y, double* p, double* q1_out, lm_step_info* info, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    LM_TRY(check_match_args(o, X, Y, p));
    if (!info) return fail(LM_EINVAL, "info is NULL");
    std::memset(info, 0, sizeof *info);
    hipStream_t st = (hipStream_t)stream;
    Workspace ws(st);
    FeedbackWork w;
    LM_TRY(w.alloc(ws, prm, n, X, st));
    LM_TRY(w.prepare_solver(ws, prm, o, n, X, st));
    EventTimer timer;
    LM_TRY(timer.init());
    LM_HIP(hipEventRecord(timer.ev[0], st));
    double r = 0.0;
    LM_TRY(feedback_shoot_residual(prm, o, n, X, Y, p, w, &r, st, timer.ev[1]));
    info->shoot_ms = timer.ms(0, 1);
    info->resid_inf = r;
    if (q1_out) LM_HIP(hipMemcpyAsync(q1_out, w.q1, (int64_t)prm->dim * n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (!is_finite(r)) return fail(LM_EDIVERGED, "non-finite residual");
    if (r < o->tol) {
        info->converged = 1;
        LM_HIP(hipStreamSynchronize(st));
        return LM_OK;
    }
    LM_HIP(hipEventRecord(timer.ev[2], st));
    int32_t cgit = 0;
    lm_status s = feedback_update(prm, o, n, X, Y, p, w, &cgit, st);
    info->cg_iters = cgit;
    LM_TRY(s);
    LM_HIP(hipEventRecord(timer.ev[3], st));
    LM_HIP(hipEventSynchronize(timer.ev[3]));
    info->solve_ms = timer.ms(2, 3);
    return LM_OK;
}

lm_status lm_velocity(const lm_params* prm, int64_t n, const void* q, const void* p, int64_t m, const void* x,
                      void* u, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    LM_TRY(check_n(m, "m"));
    if (!q || !p || !x || !u) return fail(LM_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F64)
        return velocity_t<double>(prm, n, (const double*)q, (const double*)p, m, (const double*)x, (double*)u, st);
    return velocity_t<float>(prm, n, (const float*)q, (const float*)p, m, (const float*)x, (float*)u, st);
}


lm_status lm_flow_points(const lm_params* prm, int64_t n, const void* q0, const void* p0, int64_t m, const void* x0,
                         double t1, int32_t steps, void* q1, void* p1, void* x1, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    LM_TRY(check_n(m, "m"));
    if (!q0 || !p0 || !x0 || !x1) return fail(LM_EINVAL, "NULL buffer");
    if (steps < 1) return fail(LM_EINVAL, "steps must be >= 1 (got %d)", steps);
    if (!is_finite(t1)) return fail(LM_EINVAL, "t1 must be finite");
    const size_t es = prm->dtype == LM_F64 ? sizeof(double) : sizeof(float);
    const size_t bq = (size_t)prm->dim * (size_t)n * es, bx = (size_t)prm->dim * (size_t)m * es;
    // the points must not share memory with the particles' buffers
    auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
        const char *x = (const char*)a, *y = (const char*)b;
        return a && b && x < y + nb && y < x + na;
    };
    const void* parts[4] = {q0, p0, q1, p1};
    for (const void* b : parts)
        if (overlap(x1, bx, b, bq) || overlap(x0, bx, b, bq))
            return fail(LM_EINVAL, "x0/x1 must not overlap the particle buffers");
    if ((q1 && q1 != q0 && overlap(q1, bq, q0, bq)) || (p1 && p1 != p0 && overlap(p1, bq, p0, bq)) ||
        (q1 && p1 && overlap(q1, bq, p1, bq)))
        return fail(LM_EINVAL, "q1/p1 must be q0/p0 themselves or disjoint buffers");
    hipStream_t st = (hipStream_t)stream;
    if (prm->dtype == LM_F64)
        return flow_t<double>(prm, n, (const double*)q0, (const double*)p0, m, (const double*)x0, t1, steps,
                              (double*)q1, (double*)p1, (double*)x1, st);
    return flow_t<float>(prm, n, (const float*)q0, (const float*)p0, m, (const float*)x0, t1, steps, (float*)q1,
                         (float*)p1, (float*)x1, st);
}

lm_status lm_rhs_vjp(const lm_params* prm, int64_t n, const double* q, const double* p, const double* a,
                     const double* b, double* aq, double* ap, void* stream)
{
    LM_TRY(check_adjoint_params(prm));
    LM_TRY(check_n(n));
    if (!q || !p || !a || !b || !aq || !ap) return fail(LM_EINVAL, "NULL buffer");
    const void* ins[4] = {q, p, a, b};
    for (const void* x : ins)
        if (x == aq || x == ap) return fail(LM_EINVAL, "aq/ap must not alias the inputs");
    hipStream_t st = (hipStream_t)stream;
    Workspace ws(st);
    double* part;
    LM_TRY(ws.get(&part, vjp_part_elems(prm, n)));
    lm::AdjEpi e{};
    e.kind = lm::ADJ_STORE;
    e.cscale = 1.0;
    e.tau = prm->tau;
    e.cot_q = a;
    e.lam_q = aq;
    e.lam_p = ap;
    return vjp_eval(prm, n, q, p, a, b, e, part, st);
}

lm_status lm_shoot_adjoint(const lm_params* prm, int64_t n, const double* q0, const double* p0, double t1,
                           int32_t steps, int32_t ckpt_every, const double* gq1, const double* gp1, double* gq0,
                           double* gp0, double* q1, double* p1, void* stream)
{
    LM_TRY(check_adjoint_params(prm));
    LM_TRY(check_n(n));
    if (!q0 || !p0 || !gq1 || !gp1 || !gq0 || !gp0) return fail(LM_EINVAL, "NULL buffer");
    if (steps < 1) return fail(LM_EINVAL, "steps must be >= 1");
    if (ckpt_every < 0) return fail(LM_EINVAL, "ckpt_every must be >= 0");
    if (!is_finite(t1)) return fail(LM_EINVAL, "t1 must be finite");
    hipStream_t st = (hipStream_t)stream;
    Workspace ws(st);
    AdjointWork W;
    LM_TRY(W.alloc(ws, prm, n, t1, steps, ckpt_every));
    const int64_t m = W.m;
    const double* yT = nullptr;
    LM_TRY(adjoint_forward(prm, n, q0, p0, W, &yT, st));
    if (q1) LM_HIP(hipMemcpyAsync(q1, yT, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (p1) LM_HIP(hipMemcpyAsync(p1, yT + m, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(hipMemcpyAsync(W.L0, gq1, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(hipMemcpyAsync(W.L0 + m, gp1, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    const double* lam = nullptr;
    LM_TRY(adjoint_reverse(prm, n, W, &lam, st));
    LM_HIP(hipMemcpyAsync(gq0, lam, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    LM_HIP(hipMemcpyAsync(gp0, lam + m, m * sizeof(double), hipMemcpyDeviceToDevice, st));
    return LM_OK;
}

lm_status lm_energy_grad(const lm_params* prm, int64_t n, const double* X, const double* Y, const double* p0,
                         double lam, double reg, int32_t steps, int32_t ckpt_every, double* E_out, double* grad,
                         double* q1, void* stream)
{
    LM_TRY(check_adjoint_params(prm));
    LM_TRY(check_n(n));
    if (!X || !Y || !p0 || !E_out || !grad) return fail(LM_EINVAL, "NULL pointer");
    if (!(lam >= 0.0) || !is_finite(lam) || !(reg >= 0.0) || !is_finite(reg))
        return fail(LM_EINVAL, "lam and reg must be >= 0 and finite");
    if (steps < 1 || ckpt_every < 0) return fail(LM_EINVAL, "bad steps or ckpt_every");
    if (grad == p0) return fail(LM_EINVAL, "grad must not alias p0");
    hipStream_t st = (hipStream_t)stream;
    Workspace ws(st);
    EnergyWork E;
    LM_TRY(E.alloc(ws, prm, n, steps, ckpt_every));
    return energy_grad_impl(prm, n, X, Y, p0, lam, reg, E, E_out, grad, q1, nullptr, st);
}

lm_status lm_lbfgs_match(const lm_params* prm, const lm_lbfgs_opts* o, int64_t n, const double* X, const double* Y,
                         double* p0, lm_lbfgs_info* info, void* stream)
{
    LM_TRY(check_adjoint_params(prm));
    LM_TRY(check_n(n));
    if (!o || !info || !X || !Y || !p0) return fail(LM_EINVAL, "NULL pointer");
    if (!(o->lam >= 0.0) || !(o->reg >= 0.0) || !is_finite(o->lam) || !is_finite(o->reg))
        return fail(LM_EINVAL, "lam and reg must be >= 0 and finite");
    if (o->max_iter < 0 || o->steps < 1 || o->ckpt_every < 0 || o->history < 0 || o->history > 64)
        return fail(LM_EINVAL, "bad iteration settings");
    if (!(o->gtol >= 0.0) || !(o->match_tol >= 0.0)) return fail(LM_EINVAL, "tolerances must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    std::memset(info, 0, sizeof *info);
    Workspace ws(st);
    EnergyWork EW;
    LM_TRY(EW.alloc(ws, prm, n, o->steps, o->ckpt_every));
    return lbfgs_impl(prm, o, n, X, Y, p0, info, EW, ws, st);
}

lm_status lm_shoot_noalloc(const lm_params* prm, int64_t n, const void* q0, const void* p0, double t1,
                           int32_t steps, void* q1, void* p1, void* stream)
{
    LM_TRY(check_params(prm));
    LM_TRY(check_n(n));
    if (!q0 || !p0 || !q1 || !p1) return fail(LM_EINVAL, "NULL buffer");
    if (steps < 1) return fail(LM_EINVAL, "steps must be >= 1 (got %d)", steps);
    if (!is_finite(t1)) return fail(LM_EINVAL, "t1 must be finite");
    if (q1 == p1) return fail(LM_EINVAL, "q1 and p1 must be distinct buffers");
    if (prm->cutoff > 0.0) return fail(LM_EUNSUPPORTED, "lm_shoot_noalloc sums every pair: cutoff must be 0");
    const size_t need = noalloc_bytes(prm, n);
    if (need > kScratchBytes)
        return fail(LM_ENOMEM, "lm_shoot_noalloc: n = %lld needs %zu bytes of scratch, beyond its fixed %zu bytes",
                    (long long)n, need, kScratchBytes);
    hipStream_t st = (hipStream_t)stream;
    int cur = -1;
    LM_HIP(hipGetDevice(&cur));
    if (st) {
        int sdev = -1;
        LM_HIP(hipStreamGetDevice(st, &sdev));
        if (sdev != cur) return fail(LM_EINVAL, "the stream belongs to device %d, the current device is %d", sdev, cur);
    }
    unsigned char* base = nullptr;
    LM_TRY(scratch_base(cur, &base));
    if (prm->dtype == LM_F64)
        return shoot_noalloc_t<double>(prm, n, (const double*)q0, (const double*)p0, t1, steps, (double*)q1,
                                       (double*)p1, base, st);
    return shoot_noalloc_t<float>(prm, n, (const float*)q0, (const float*)p0, t1, steps, (float*)q1, (float*)p1,
                                  base, st);
}

}  // extern "C"
