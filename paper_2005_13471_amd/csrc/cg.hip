// Conjugate gradients on the normal equations (H^T H) x = b (Sec. 2: one
// back projection, then the Gram filter in every iteration).  Vectors live in
// the working precision; every inner product and the residual norm are
// accumulated in FP64.  All scalars stay on the device, so a chunk of
// iterations is queued without host round trips; the host reads the state
// once per chunk.  Once converged (or broken down) the status word is set
// and every kernel queued after it returns at once.
//
// An iteration is three kernels, the Gram-filtering passes with the vector
// work folded in (gram_apply.hip, k_cgf_*), in the Chronopoulos-Gear
// arrangement: the inverse row pass forms w = A r and the FP64 partial dots
// r.r and r.w; the next forward row pass reduces them, derives beta and
// alpha, updates p, s = A p, x and r on its rows and transforms the new r.
// In exact arithmetic these are the textbook CG iterates.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "gct_internal.h"

namespace gct {

int apply_row_blocks(const gct_plan *p, size_t elem);

constexpr int VBLK = 256;  // blocks of the vector kernels (fixed: deterministic reductions)

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// r = b - Ax (or b), p = r, x = 0 when no start vector; partial ||r||^2, ||b||^2.
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_init(const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r, T *__restrict__ p,
          const T *__restrict__ Ax, size_t n, double *__restrict__ part_rr,
          double *__restrict__ part_bb)
{
    double rr = 0.0, bb = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const T bi = b[i];
        T ri;
        if (Ax) {
            ri = bi - Ax[i];
        } else {
            ri = bi;
            x[i] = T(0);
        }
        r[i] = ri;
        p[i] = ri;
        rr += (double)ri * (double)ri;
        bb += (double)bi * (double)bi;
    }
    rr = block_sum(rr);
    bb = block_sum(bb);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = rr;
        part_bb[blockIdx.x] = bb;
    }
}

__global__ void __launch_bounds__(256)
k_cg_init_fin(CGState *st, const double *part_rr, const double *part_bb, int np, double rtol2, int sd)
{
    double rr = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        rr += part_rr[i];
        bb += part_bb[i];
    }
    rr = block_sum(rr);
    bb = block_sum(bb);
    if (threadIdx.x == 0) {
        st->rr = rr;
        st->bb = bb;
        st->rr0 = rr;
        st->beta = 0.0;
        st->thr2 = rtol2 * bb;
        st->k = 0;
        st->ring[0] = rr;
        st->status = (rr <= st->thr2) ? CG_CONVERGED : CG_RUNNING;
        if (!(rr == rr) || !(bb == bb)) st->status = CG_BREAKDOWN;
        st->gam[0] = st->gam[1] = rr;
        st->alp[0] = st->alp[1] = 1.0;
        st->pend[0] = st->pend[1] = 0;
        st->stat[0] = st->stat[1] = st->status;
        st->kring = 0;
        st->sd = sd;
        st->fb = 0;
    }
}

// Start-vector fallback on the device: if ||b - A x_0|| >= ||b|| (or is not
// finite) the solve starts from zero instead.  Vector part (every block),
// then the scalars (one block); both read the decision from the state that
// k_cg_init_fin wrote, which neither changes before the second kernel.
__device__ __forceinline__ bool cg_drop_start(const CGState *st)
{
    return st->bb > 0.0 && !(st->rr0 < st->bb);
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_fallback_vec(const CGState *st, const T *b, T *x, T *r, size_t n)
{
    if (!cg_drop_start(st)) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        x[i] = T(0);
        r[i] = b[i];
    }
}

__global__ void k_cg_fallback_fin(CGState *st)
{
    if (threadIdx.x != 0 || !cg_drop_start(st)) return;
    const double bb = st->bb;
    st->rr = st->rr0 = bb;
    st->ring[0] = bb;
    st->status = (bb <= st->thr2) ? CG_CONVERGED : CG_RUNNING;
    st->gam[0] = st->gam[1] = bb;
    st->stat[0] = st->stat[1] = st->status;
    st->fb = 1;
}

// After the last launch of a solve that reached max_iter: ||r_k||^2 from the
// last inverse row pass's partials (the norm the next launch would test),
// recorded and tested against the stopping rule.
__global__ void __launch_bounds__(256) k_cgf_norm(CGState *st, const double *part, int np)
{
    if (st->status != CG_RUNNING) return;
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        st->ring[st->k % CG_RING] = s;
        st->kring = st->k;
        st->rr = s;
        if (!(s == s)) st->status = CG_BREAKDOWN;
        else if (s <= st->thr2) st->status = CG_CONVERGED;
    }
}

// The solver state copied to the pinned host buffer by the GPU itself (plain
// vector stores over the host link, then a system-scope fence): no copy
// engine in the host's check of a chunk.
__global__ void __launch_bounds__(64) k_state_out(const CGState *st, CGState *out)
{
    constexpr int nw = (int)(sizeof(CGState) / sizeof(int64_t));
    static_assert(sizeof(CGState) % sizeof(int64_t) == 0, "state words");
    const int64_t *src = reinterpret_cast<const int64_t *>(st);
    int64_t *dst = reinterpret_cast<int64_t *>(out);
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
    __threadfence_system();
}

// Waits for an event by polling it (no sleep between polls: a chunk ends
// within microseconds of the check, and a yielding wait adds its wake-up
// latency to every check).
static hipError_t spin_wait(hipEvent_t e)
{
    for (;;) {
        const hipError_t q = hipEventQuery(e);
        if (q != hipErrorNotReady) return q;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill_one(T *v, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        v[i] = T(1);
}

// partial ||b - Ax||^2
template <typename T>
__global__ void __launch_bounds__(256)
k_resid(const T *__restrict__ b, const T *__restrict__ Ax, size_t n, double *__restrict__ part)
{
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double d = (double)b[i] - (double)Ax[i];
        acc += d * d;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256) k_sum(const double *part, int np, double *out)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
struct CGLayout {
    size_t apply, r, p, Ap, sv, xt, part, part2, st, total;
};

static CGLayout cg_layout(const gct_plan *p, size_t elem)
{
    CGLayout L;
    const size_t img = align256((size_t)p->N * p->N * elem);
    const int np = std::max(VBLK, apply_row_blocks(p, elem));
    size_t o = 0;
    L.apply = o; o += apply_ws_bytes(p, elem);
    L.r = o; o += img;
    L.p = o; o += img;
    L.Ap = o; o += img;
    L.sv = o; o += img;  // s = A p of the fused iteration
    L.xt = o; o += img;  // iterate of the autotuner's trial solves
    L.part = o; o += align256((size_t)2 * np * sizeof(double));  // r.r and r.w per row pair
    L.part2 = o; o += align256((size_t)np * sizeof(double));
    L.st = o; o += align256(sizeof(CGState));
    L.total = o;
    return L;
}

size_t cg_ws_bytes(const gct_plan *p, size_t elem) { return cg_layout(p, elem).total; }

#define GCT_TRY(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return check_hip(e_, #call);   \
    } while (0)

// ---------------------------------------------------------------------------
// Graph cache: a chunk of CG iterations captured as a hipGraph, keyed by the
// buffers it touches, kept in the plan until it is destroyed.  Capture runs
// on a private non-blocking stream of default priority.
// ---------------------------------------------------------------------------
static hipGraphExec_t cg_graph_lookup(const gct_plan *p, const CGGraphKey &k)
{
    for (const auto &e : p->cg_graphs)
        if (e.key == k) return e.exec;
    return nullptr;
}

static void cg_graph_store(const gct_plan *p, const CGGraphKey &k, hipGraphExec_t exec)
{
    auto &v = const_cast<gct_plan *>(p)->cg_graphs;
    if (v.size() >= 16) {
        (void)hipGraphExecDestroy(v.front().exec);
        v.erase(v.begin());
    }
    v.push_back({k, exec});
}

static hipStream_t cg_capture_stream(const gct_plan *p)
{
    gct_plan *q = const_cast<gct_plan *>(p);
    if (!q->capture_stream &&
        hipStreamCreateWithFlags(&q->capture_stream, hipStreamNonBlocking) != hipSuccess)
        q->capture_stream = nullptr;
    return q->capture_stream;
}

// One solve from x (or zero) until the recursive residual meets rtol, the
// iterations run out or the recurrence breaks down; the true residual of the
// returned iterate is recomputed at the end.
template <typename T>
static int cg_run(const gct_plan *p, const T *Ghat, const T *b, T *x, int use_x0, double rtol,
                  int max_iter, int check_every, double *hist, gct_cg_result *res, void *ws,
                  hipStream_t s, int method)
{
    const CGLayout L = cg_layout(p, sizeof(T));
    char *w = reinterpret_cast<char *>(ws);
    void *aws = w + L.apply;
    T *r = reinterpret_cast<T *>(w + L.r), *pv = reinterpret_cast<T *>(w + L.p);
    T *Ap = reinterpret_cast<T *>(w + L.Ap);
    T *sv = reinterpret_cast<T *>(w + L.sv);
    double *part = reinterpret_cast<double *>(w + L.part);
    double *part2 = reinterpret_cast<double *>(w + L.part2);
    CGState *st = reinterpret_cast<CGState *>(w + L.st);
    const size_t n = (size_t)p->N * p->N;
    const int rblocks = apply_row_blocks(p, sizeof(T));
    if (check_every <= 0) check_every = 8;
    if (check_every > CG_RING) check_every = CG_RING;
    check_every += check_every & 1;  // even chunks keep the parity slots aligned across replays

    // pinned state copy and its event (once per plan)
    gct_plan *pm = const_cast<gct_plan *>(p);
    if (!pm->cg_pin) {
        void *h = nullptr;
        // coherent: the GPU writes it directly (k_state_out)
        GCT_TRY(hipHostMalloc(&h, sizeof(CGState), hipHostMallocCoherent));
        pm->cg_pin = reinterpret_cast<CGState *>(h);
    }
    if (!pm->cg_ev) GCT_TRY(hipEventCreateWithFlags(&pm->cg_ev, hipEventDisableTiming));
    CGState *pin = pm->cg_pin;

    // start: r_0 (from x_0 when given), then on the device the fallback to
    // zero when x_0 is no better; no host round trip before the iterations
    if (use_x0) GCT_TRY(launch_gram_apply<T>(p, Ghat, x, Ap, aws, s));
    hipLaunchKernelGGL(k_cg_init<T>, dim3(VBLK), dim3(256), 0, s, b, x, r, pv, use_x0 ? (const T *)Ap : nullptr,
                       n, part, part2);
    hipLaunchKernelGGL(k_cg_init_fin, dim3(1), dim3(256), 0, s, st, part, part2, VBLK, rtol * rtol,
                       method == 1 ? 1 : 0);
    if (use_x0) {
        hipLaunchKernelGGL(k_cg_fallback_vec<T>, dim3(VBLK), dim3(256), 0, s, (const CGState *)st, b, x, r, n);
        hipLaunchKernelGGL(k_cg_fallback_fin, dim3(1), dim3(64), 0, s, st);
    }
    GCT_TRY(hipGetLastError());

    // launch i (of a batch starting at launch `first`): three fused kernels,
    // parity (first + i) & 1; launch 0 only forms A r_0, launch i > 0 makes
    // update i - 1, so max_iter updates take max_iter + 1 launches
    auto launch_iters = [&](int count, int64_t first, hipStream_t st_) -> hipError_t {
        for (int i = 0; i < count; ++i) {
            hipError_t e = launch_cgf_iteration<T>(p, Ghat, x, r, pv, sv, Ap, aws, part, st,
                                                   (int)((first + i) & 1), st_);
            if (e != hipSuccess) return e;
        }
        return hipGetLastError();
    };
    // one chunk of launches (a graph of check_every launches, captured once
    // per buffer set, or a shorter tail), then the state copied to the
    // pinned buffer
    const int64_t launches = max_iter > 0 ? (int64_t)max_iter + 1 : 0;
    int64_t launched = 0;
    auto enqueue = [&]() -> int {
        const int chunk = (int)std::min<int64_t>(check_every, launches - launched);
        if (chunk == check_every) {
            const CGGraphKey key{(const void *)Ghat, (void *)x, ws, (int)sizeof(T), chunk};
            hipGraphExec_t exec = cg_graph_lookup(p, key);
            if (!exec) {
                hipStream_t cs = cg_capture_stream(p);
                if (!cs) return fail(GCT_EHIP, "cannot create the capture stream");
                hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) return check_hip(e, "cg graph capture");
                e = launch_iters(chunk, 0, cs);  // replayed at even `launched` only
                hipGraph_t g = nullptr;
                hipError_t e2 = hipStreamEndCapture(cs, &g);
                if (e != hipSuccess || e2 != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return check_hip(e != hipSuccess ? e : e2, "cg graph capture");
                }
                e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return check_hip(e, "hipGraphInstantiate");
                cg_graph_store(p, key, exec);
            }
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) return check_hip(e, "cg chunk launch");
        } else {
            hipError_t e = launch_iters(chunk, launched, s);
            if (e != hipSuccess) return check_hip(e, "cg chunk launch");
        }
        launched += chunk;
        hipLaunchKernelGGL(k_state_out, dim3(1), dim3(64), 0, s, (const CGState *)st, pin);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(pm->cg_ev, s);
        return check_hip(e, "cg state copy");
    };
    CGState hs;
    int rc = GCT_OK;
    if (launches == 0) {  // no iteration: the state after the start
        GCT_TRY(hipMemcpyAsync(pin, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
        GCT_TRY(hipStreamSynchronize(s));
        hs = *pin;
    } else {
        // one chunk at a time: a chunk queued ahead of the check would run
        // (skipping) after convergence and delay the true-residual step more
        // than the overlapped check saves
        if ((rc = enqueue()) != GCT_OK) return rc;
        int64_t kprev = 0;
        bool first = true;
        for (;;) {
            GCT_TRY(spin_wait(pm->cg_ev));
            std::atomic_thread_fence(std::memory_order_acquire);
            hs = *pin;
            if (first) {
                if (hist) hist[0] = hs.bb > 0.0 ? std::sqrt(hs.rr0 / hs.bb) : 0.0;
                first = false;
            }
            if (hist)
                for (int64_t k = kprev + 1; k <= hs.kring; ++k)
                    hist[k] = hs.bb > 0.0 ? std::sqrt(hs.ring[k % CG_RING] / hs.bb) : 0.0;
            kprev = std::max(kprev, hs.kring);
            if (hs.status != CG_RUNNING || launched >= launches) break;
            if ((rc = enqueue()) != GCT_OK) return rc;
        }
    }
    const double bb = hs.bb;
    auto rel = [bb](double rr) { return bb > 0.0 ? std::sqrt(rr / bb) : 0.0; };
    res->rel_res0 = rel(hs.rr0);
    res->fell_back = (int32_t)hs.fb;
    if (hist && launches == 0) hist[0] = rel(hs.rr0);
    const int64_t done = launched;
    if (hs.status == CG_RUNNING && done > 0) {
        // max_iter updates made: test the last residual norm
        hipLaunchKernelGGL(k_cgf_norm, dim3(1), dim3(256), 0, s, st, (const double *)part, rblocks);
        GCT_TRY(hipGetLastError());
        const int64_t kprev = hs.kring;
        GCT_TRY(hipMemcpyAsync(pin, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
        GCT_TRY(hipStreamSynchronize(s));
        hs = *pin;
        if (hist)
            for (int64_t k = kprev + 1; k <= hs.kring; ++k) hist[k] = rel(hs.ring[k % CG_RING]);
    }
    // true residual of the returned iterate
    GCT_TRY(launch_gram_apply<T>(p, Ghat, x, Ap, aws, s));
    hipLaunchKernelGGL(k_resid<T>, dim3(VBLK), dim3(256), 0, s, b, Ap, n, part);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, part, VBLK, &st->pad);
    hipLaunchKernelGGL(k_state_out, dim3(1), dim3(64), 0, s, (const CGState *)st, pin);
    GCT_TRY(hipGetLastError());
    GCT_TRY(hipEventRecord(pm->cg_ev, s));
    GCT_TRY(spin_wait(pm->cg_ev));
    std::atomic_thread_fence(std::memory_order_acquire);
    const double rt = pin->pad;

    res->iters = (int32_t)hs.k;
    res->rel_res = rel(hs.rr);
    res->rel_res_true = rel(rt);
    if (hs.status == CG_CONVERGED) res->status = GCT_OK;
    else if (hs.status == CG_BREAKDOWN) res->status = GCT_EBREAKDOWN;
    else res->status = GCT_ENOTCONV;
    return res->status;
}

// Restarts after the recursive residual met the rule while the recomputed
// one did not (at most this many, within max_iter in total).
constexpr int CG_MAX_RESTARTS = 4;

// The solver: GCT_OK only when the recomputed residual ||b - A x||/||b|| of
// the returned iterate is within rtol.  The recursive residual drifts from
// the true one by rounding; when it meets the rule alone, CG restarts from
// the current iterate with r = b - A x (residual replacement), continuing
// the iteration count and the history.
template <typename T>
int cg_solve(const gct_plan *p, const T *Ghat, const T *b, T *x, int use_x0, double rtol,
             int max_iter, int check_every, double *hist, gct_cg_result *res, void *ws,
             hipStream_t s, int method)
{
    int64_t done = 0;
    for (int run = 0;; ++run) {
        gct_cg_result r{};
        const int left = (int)(max_iter - done);
        const int rc = cg_run<T>(p, Ghat, b, x, use_x0 || run > 0, rtol, left, check_every,
                                 hist ? hist + done : nullptr, &r, ws, s, method);
        if (rc != GCT_OK && rc != GCT_ENOTCONV && rc != GCT_EBREAKDOWN) return rc;
        if (run == 0) {
            res->rel_res0 = r.rel_res0;
            res->fell_back = r.fell_back;
        }
        done += r.iters;
        res->iters = (int32_t)done;
        res->rel_res = r.rel_res;
        res->rel_res_true = r.rel_res_true;
        res->status = r.status;
        if (r.status == GCT_OK && !(r.rel_res_true <= rtol)) {
            if (done < max_iter && run < CG_MAX_RESTARTS) continue;
            res->status = GCT_ENOTCONV;
        }
        return res->status;
    }
}

// Times the apply passes for every candidate pair (row passes E, column
// pass Ec; apply_e_ok) on zero input in the CG workspace's vectors and keeps
// the fastest for this dtype; then the same for the fused CG passes, on
// trial solves.  Each candidate's launches are captured as one graph and the
// best of a few replays is kept, so host launch overhead and one-off noise
// do not decide.  Cached CG graphs (built with the old tiling) are dropped.
template <typename T>
int plan_autotune(gct_plan *p, const T *Ghat, void *ws, int reps, int32_t *chosen, hipStream_t s)
{
    const CGLayout L = cg_layout(p, sizeof(T));
    char *w = reinterpret_cast<char *>(ws);
    T *src = reinterpret_cast<T *>(w + L.r), *dst = reinterpret_cast<T *>(w + L.Ap);
    T *sv = reinterpret_cast<T *>(w + L.sv), *pv = reinterpret_cast<T *>(w + L.p);
    T *xt = reinterpret_cast<T *>(w + L.xt);
    double *part = reinterpret_cast<double *>(w + L.part);
    double *part2 = reinterpret_cast<double *>(w + L.part2);
    CGState *st = reinterpret_cast<CGState *>(w + L.st);
    void *aws = w + L.apply;
    const int t = sizeof(T) == 4 ? 0 : 1;
    const size_t n = (size_t)p->N * p->N;
    reps += reps & 1;  // even: the CG parity slots line up across replays
    hipStream_t cs = cg_capture_stream(p);
    if (!cs) return fail(GCT_EHIP, "cannot create the capture stream");
    GCT_TRY(hipMemsetAsync(src, 0, n * sizeof(T), s));
    hipEvent_t e0, e1;
    GCT_TRY(hipEventCreate(&e0));
    GCT_TRY(hipEventCreate(&e1));
    hipError_t err = hipSuccess;
    // best of three replays of the graph of `body` (launches on the capture
    // stream); `prep` (launches on s) runs before each replay, untimed
    auto time_graph = [&](auto body, auto prep) -> float {
        float best = 1e30f;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (err != hipSuccess) return best;
        hipError_t eb = body(cs);
        err = hipStreamEndCapture(cs, &g);
        if (err == hipSuccess) err = eb;
        if (err == hipSuccess) err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
            prep();
            err = hipGetLastError();
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            if (err == hipSuccess) err = hipGraphLaunch(ge, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess && rep > 0) best = std::min(best, ms);  // replay 0 warms up
        }
        if (ge) (void)hipGraphExecDestroy(ge);
        return best;
    };
    // candidate elements per thread: 16, 8, 4 (powers of two), 24, 12 (three times a power of two)
    const int c3 = p->P % 3 == 0;
    auto cand = [c3](int i) { return c3 ? (i == 0 ? 24 : (i == 1 ? 12 : 0)) : 16 >> i; };
    int best = p->fft_e[t], best_c = p->fft_ec[t];
    float best_ms = 1e30f;
    for (int pr = 0; pr < 9 && err == hipSuccess; ++pr) {
        const int E = cand(pr / 3), Ec = cand(pr % 3);
        if (!apply_e_ok(p->pc, E) || !apply_e_ok(p->pc, Ec)) continue;
        p->fft_e[t] = E;
        p->fft_ec[t] = Ec;
        const float ms = time_graph(
            [&](hipStream_t q) {
                for (int r = 0; r < reps; ++r) {
                    hipError_t e = launch_gram_apply<T>(p, Ghat, src, dst, aws, q);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            },
            [] {});
        if (err == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = E;
            best_c = Ec;
        }
    }
    p->fft_e[t] = best;
    p->fft_ec[t] = best_c;
    // the fused CG passes: a trial solve of A x = 1 that never meets its
    // stopping rule (rtol = 0), restarted before each replay of `reps`
    // iterations
    int best_cg = p->cg_e[t], best_cgc = p->cg_ec[t];
    float best_cg_ms = 1e30f;
    for (int pr = 0; pr < 9 && err == hipSuccess; ++pr) {
        const int E = cand(pr / 3), Ec = cand(pr % 3);
        if (!apply_e_ok(p->pc, E) || !apply_e_ok(p->pc, Ec)) continue;
        p->cg_e[t] = E;
        p->cg_ec[t] = Ec;
        const float ms = time_graph(
            [&](hipStream_t q) {
                for (int it = 0; it < reps; ++it) {
                    hipError_t e = launch_cgf_iteration<T>(p, Ghat, xt, src, pv, sv, dst, aws, part, st, it & 1, q);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            },
            [&] {
                hipLaunchKernelGGL(k_fill_one<T>, dim3(VBLK), dim3(256), 0, s, sv, n);
                hipLaunchKernelGGL(k_cg_init<T>, dim3(VBLK), dim3(256), 0, s, (const T *)sv, xt, src, pv, nullptr,
                                   n, part, part2);
                hipLaunchKernelGGL(k_cg_init_fin, dim3(1), dim3(256), 0, s, st, part, part2, VBLK, 0.0, 0);
            });
        if (err == hipSuccess && ms < best_cg_ms) {
            best_cg_ms = ms;
            best_cg = E;
            best_cgc = Ec;
        }
    }
    p->cg_e[t] = best_cg;
    p->cg_ec[t] = best_cgc;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return check_hip(err, "plan autotune");
    for (auto &g : p->cg_graphs) (void)hipGraphExecDestroy(g.exec);
    p->cg_graphs.clear();
    if (chosen) *chosen = best;
    return GCT_OK;
}

template int plan_autotune<float>(gct_plan *, const float *, void *, int, int32_t *, hipStream_t);
template int plan_autotune<double>(gct_plan *, const double *, void *, int, int32_t *, hipStream_t);

template int cg_solve<float>(const gct_plan *, const float *, const float *, float *, int, double,
                             int, int, double *, gct_cg_result *, void *, hipStream_t, int);
template int cg_solve<double>(const gct_plan *, const double *, const double *, double *, int,
                              double, int, int, double *, gct_cg_result *, void *, hipStream_t, int);

}  // namespace gct
