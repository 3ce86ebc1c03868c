// Batched uneven slices: many independent slices (each with its own plan:
// N, angle set, blur) run through Gram-filter construction, Gram filtering
// and CG together.  Every phase is ONE launch over all slices (per FFT size
// for the transform passes), indexed through a block -> (slice, local index)
// map, so the whole batch fills the GPU even when single slices cannot.
// CG keeps per-slice state and status words: converged slices drop out
// while the others continue; chunks of iterations are replayed as a hipGraph.
// An autotuner picks, per FFT size, the elements per thread of the
// transforms (the shape of the work tile) by timing the batched apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fft_passes.h"

namespace gct {

template <typename T>
hipError_t launch_batch_gram_build(const int2 *map, int nblocks, const BatchSlice *sl, T *G,
                                   hipStream_t s);

constexpr int BVB = 8;  // vector-kernel blocks per slice
constexpr int BATCH_MAX_RESTARTS = 4;

__device__ __forceinline__ bool slice_halted(const CGState *st, int s)
{
    return st && st[s].status != CG_RUNNING;
}

// ---------------------------------------------------------------------------
// Batched transform passes
// ---------------------------------------------------------------------------
template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
kb_rows_fwd(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
            const T *__restrict__ src, C2<T> *__restrict__ W1, const CGState *st, T *pupd)
{
    const int2 m = map[xcd_swizzle(blockIdx.x, gridDim.x)];
    if (slice_halted(st, m.x)) return;
    const BatchSlice &d = sl[m.x];
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    // data first, then the twiddles: their latencies overlap
    C2<T> v[E];
    rows_fwd_load<T, PC, E>(2 * m.y, src + d.img, d.N, pupd ? pupd + d.img : nullptr,
                              pupd ? (T)st[m.x].beta : T(0), v);
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), reinterpret_cast<const C2<T> *>(d.tw));
    __syncthreads();
    rows_fwd_regs<T, PC, E>(2 * m.y, v, W1 + d.w, d.N, x, tws);
}

// Two row pairs per block (rows 4j .. 4j+3 of a slice), for the long
// transforms: each group of G = P/E threads transforms one pair as above,
// then the block writes the four rows' spectra column by column with
// neighbouring lanes on neighbouring pairs, so each column gets one 32-byte
// run per block instead of two 16-byte ones (the transposed scratch is
// written a few bytes per cache line; fewer, larger requests move it
// faster).  FP32 with even N (paired 16-byte accesses).
template <typename T, int PC, int E>
__global__ void __launch_bounds__(512)
kb_rows_fwd2(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
             const T *__restrict__ src, C2<T> *__restrict__ W1, const CGState *st, T *pupd)
{
    constexpr int P = fft_size(PC), hP = P / 2, G = P / E;
    const int2 m = map[xcd_swizzle(blockIdx.x, gridDim.x)];
    if (slice_halted(st, m.x)) return;
    const BatchSlice &d = sl[m.x];
    const int N = d.N;
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *xs = reinterpret_cast<C2<T> *>(smem_raw);
    C2<T> *x = xs + grp * P;
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), hP, 2 * G>(xs + 2 * P, reinterpret_cast<const C2<T> *>(d.tw));
    __syncthreads();
    const int ra = 4 * m.y + 2 * grp, rb = ra + 1;
    const T *sr = src + d.img;
    T *pu = pupd ? pupd + d.img : nullptr;
    const T bt = pupd ? (T)st[m.x].beta : T(0);
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = t + G * q;
        T re = 0, im = 0;
        // q >= E/2: n >= P/2 >= N, zero padding known at compile time
        if (q < E / 2 && n < N && ra < N) {  // N even: rb < N too
            const size_t ia = (size_t)ra * N + n, ib = (size_t)rb * N + n;
            re = sr[ia];
            im = sr[ib];
            if (pu) {
                re += bt * pu[ia];
                pu[ia] = re;
                im += bt * pu[ib];
                pu[ib] = im;
            }
        }
        v[q] = {re, im};
    }
    fft_passes<T, E, P, 1, false, true, false>(v, x, t, tws);  // one area per group
#pragma unroll
    for (int q = 0; q < E; ++q) x[t + G * q] = v[q];
    __syncthreads();
    // split each pair's transform into its two real rows (as rows_fwd_regs)
    // and write (k, pair) with the pair fastest
    C2<T> *out = W1 + d.w;
    for (int i = threadIdx.x; i < 2 * (hP + 1); i += 2 * G) {
        const int k = i >> 1, g2 = i & 1, r0 = 4 * m.y + 2 * g2;
        if (r0 >= N) continue;
        const C2<T> *xg = xs + g2 * P;
        const C2<T> Zk = xg[k], Zm = xg[(P - k) % P];
        const C2<T> a = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        const C2<T> b = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
        store_pair(out + (size_t)k * N + r0, a, b);
    }
}

// Inverse rows for two row pairs per block: the block reads the four rows'
// spectra column by column (32-byte runs, pair fastest) into LDS, then each
// group transforms its pair as the single-pair inverse row pass; FP64 partial dot of the block
// in the slot of its first pair (the second pair's slot holds 0).
template <typename T, int PC, int E>
__global__ void __launch_bounds__(512)
kb_rows_inv2(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
             const C2<T> *__restrict__ W2, T *__restrict__ y, const CGState *st,
             const T *__restrict__ dotv, double *__restrict__ partial)
{
    constexpr int P = fft_size(PC), hP = P / 2, G = P / E, XS = P + 2;  // per-group area (spectra + 2)
    const int2 m = map[xcd_swizzle(blockIdx.x, gridDim.x)];
    if (slice_halted(st, m.x)) return;
    const BatchSlice &d = sl[m.x];
    const int N = d.N;
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *xs = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), hP, 2 * G>(xs + 2 * XS, reinterpret_cast<const C2<T> *>(d.tw));
    // stage: group g2's area holds (Ya, Yb) of column k at 2k, 2k + 1
    const C2<T> *in = W2 + d.w;
    for (int i = threadIdx.x; i < 2 * (hP + 1); i += 2 * G) {
        const int k = i >> 1, g2 = i & 1, r0 = 4 * m.y + 2 * g2;
        C2<T> a = {T(0), T(0)}, b = {T(0), T(0)};
        if (r0 < N) load_pair(in + (size_t)k * N + r0, a, b);
        C2<T> *sg = xs + g2 * XS;
        sg[2 * k] = a;
        sg[2 * k + 1] = b;
    }
    __syncthreads();
    const C2<T> *sg = xs + grp * XS;
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int k = t + G * q;
        const int kk = k <= hP ? k : P - k;  // Hermitian extension
        C2<T> Ya = sg[2 * kk], Yb = sg[2 * kk + 1];
        if (k > hP) {
            Ya.y = -Ya.y;
            Yb.y = -Yb.y;
        }
        v[q] = {Ya.x - Yb.y, Ya.y + Yb.x};
    }
    __syncthreads();  // the staged spectra are read: the transform may reuse the area
    fft_passes<T, E, P, 1, true, true, false>(v, xs + grp * XS, t, tws);  // one area per group
    const int ra = 4 * m.y + 2 * grp, rb = ra + 1;
    T *yo = y + d.img;
    const T *dv = dotv ? dotv + d.img : nullptr;
    double acc = 0.0;
    if (ra < N) {
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {  // n >= P/2 >= N for q >= E/2
            const int n = t + G * q;
            if (n >= N) continue;
            yo[(size_t)ra * N + n] = v[q].x;
            yo[(size_t)rb * N + n] = v[q].y;
            if (dv) {
                acc += (double)dv[(size_t)ra * N + n] * (double)v[q].x;
                acc += (double)dv[(size_t)rb * N + n] * (double)v[q].y;
            }
        }
    }
    if (partial) {
        const double sum = block_sum_lds(acc, reinterpret_cast<double *>(smem_raw));
        if (threadIdx.x == 0) {
            partial[d.rpart + 2 * m.y] = sum;
            if (2 * m.y + 1 < d.nrow) partial[d.rpart + 2 * m.y + 1] = 0.0;
        }
    }
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
kb_cols(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
        const C2<T> *__restrict__ W1, C2<T> *__restrict__ W2, const T *__restrict__ Ghat,
        const CGState *st)
{
    const int2 m = map[blockIdx.x];
    if (slice_halted(st, m.x)) return;
    const BatchSlice &d = sl[m.x];
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    C2<T> v[E];
    T gs[E];
    cols_load<T, PC, E>(m.y, W1 + d.w, Ghat + d.spec, d.N, v, gs);
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), reinterpret_cast<const C2<T> *>(d.tw));
    __syncthreads();
    cols_regs<T, PC, E>(m.y, v, gs, W2 + d.w, d.N, x, tws);
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
kb_rows_inv(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
            const C2<T> *__restrict__ W2, T *__restrict__ y, const CGState *st,
            const T *__restrict__ dotv, double *__restrict__ partial)
{
    const int2 m = map[xcd_swizzle(blockIdx.x, gridDim.x)];
    if (slice_halted(st, m.x)) return;
    const BatchSlice &d = sl[m.x];
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    C2<T> v[E];
    rows_inv_load<T, PC, E>(2 * m.y, W2 + d.w, d.N, v);
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), reinterpret_cast<const C2<T> *>(d.tw));
    __syncthreads();
    fft_passes<T, E, P, 1, true, true>(v, x, threadIdx.x, tws);
    const double acc = rows_inv_store<T, PC, E>(2 * m.y, v, y + d.img, d.N, dotv ? dotv + d.img : nullptr);
    if (partial) {
        const double s = block_sum_lds(acc, reinterpret_cast<double *>(smem_raw));
        if (threadIdx.x == 0) partial[d.rpart + m.y] = s;
    }
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
kb_spec_rows(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
             const T *__restrict__ G, C2<T> *__restrict__ R)
{
    const int2 m = map[xcd_swizzle(blockIdx.x, gridDim.x)];
    const BatchSlice &d = sl[m.x];
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), reinterpret_cast<const C2<T> *>(d.tw));
    __syncthreads();
    // R of a slice uses (P/2+1) P complex, i.e. 2 d.spec reals' worth of offset
    body_spec_rows<T, PC, E>(m.y, G + d.gram, R + d.spec, d.N, x, tws);
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
kb_spec_cols(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl,
             const C2<T> *__restrict__ R, T *__restrict__ Ghat)
{
    const int2 m = map[blockIdx.x];
    const BatchSlice &d = sl[m.x];
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws =
        stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), reinterpret_cast<const C2<T> *>(d.tw));
    __syncthreads();
    body_spec_cols<T, PC, E>(m.y, R + d.spec, Ghat + d.spec, x, tws,
                               T(1.0 / ((double)P * (double)P)));
}

// ---------------------------------------------------------------------------
// Batched CG vector kernels: BVB blocks per slice, one block per slice for
// the scalar steps.  Reductions run in a fixed order (deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bsum(double v)
{
    __shared__ double red[256];
    return block_sum_lds(v, red);
}

// r = b - A x (Ax given: start vector) or r = b, x = 0; p = r; partial
// ||r||^2 and ||b||^2 per (slice, block).
template <typename T>
__global__ void __launch_bounds__(256)
kb_cg_init(const BatchSlice *__restrict__ sl, const T *__restrict__ b, T *__restrict__ x,
           T *__restrict__ r, T *__restrict__ p, const T *__restrict__ Ax, double *__restrict__ prr,
           double *__restrict__ pbb)
{
    const int s = blockIdx.x / BVB, j = blockIdx.x % BVB;
    const BatchSlice &d = sl[s];
    const size_t n = (size_t)d.N * d.N;
    double rr = 0.0, bb = 0.0;
    for (size_t i = (size_t)j * blockDim.x + threadIdx.x; i < n; i += (size_t)BVB * blockDim.x) {
        const size_t g = d.img + i;
        const T bi = b[g];
        T ri = bi;
        if (Ax) ri = bi - Ax[g];
        else x[g] = T(0);
        r[g] = ri;
        p[g] = ri;
        rr += (double)ri * (double)ri;
        bb += (double)bi * (double)bi;
    }
    rr = bsum(rr);
    bb = bsum(bb);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = rr;
        pbb[blockIdx.x] = bb;
    }
}

// Per slice: the start's residual norm, ||b||, the stopping threshold; with
// a start vector, the fallback to zero when ||b - A x_0|| >= ||b|| (or is
// not finite), as in the single-slice solver (fb = 1: kb_cg_fallback_vec
// resets the vectors).
__global__ void __launch_bounds__(256)
kb_cg_init_fin(CGState *st, const double *prr, const double *pbb, double rtol2, int use_x0)
{
    const int s = blockIdx.x;
    const double rr_ = bsum(threadIdx.x < BVB ? prr[s * BVB + threadIdx.x] : 0.0);
    const double bb = bsum(threadIdx.x < BVB ? pbb[s * BVB + threadIdx.x] : 0.0);
    if (threadIdx.x == 0) {
        CGState &c = st[s];
        const bool drop = use_x0 && bb > 0.0 && !(rr_ < bb);
        const double rr = drop ? bb : rr_;
        c.rr = rr;
        c.bb = bb;
        c.rr0 = rr;
        c.beta = 0.0;
        c.thr2 = rtol2 * bb;
        c.k = 0;
        c.ring[0] = rr;
        c.fb = drop ? 1 : 0;
        c.status = (rr <= c.thr2) ? CG_CONVERGED : CG_RUNNING;
        if (!(rr == rr) || !(bb == bb)) c.status = CG_BREAKDOWN;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
kb_cg_fallback_vec(const CGState *st, const BatchSlice *__restrict__ sl, const T *__restrict__ b,
                   T *__restrict__ x, T *__restrict__ r, T *__restrict__ p)
{
    const int s = blockIdx.x / BVB, j = blockIdx.x % BVB;
    if (!st[s].fb) return;
    const BatchSlice &d = sl[s];
    const size_t n = (size_t)d.N * d.N;
    for (size_t i = (size_t)j * blockDim.x + threadIdx.x; i < n; i += (size_t)BVB * blockDim.x) {
        const size_t g = d.img + i;
        x[g] = T(0);
        r[g] = b[g];
        p[g] = b[g];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
kb_cg_update(CGState *st, const BatchSlice *__restrict__ sl, T *__restrict__ x,
             T *__restrict__ r, const T *__restrict__ p, const T *__restrict__ Ap,
             const double *__restrict__ rpart, double *__restrict__ upart)
{
    const int s = blockIdx.x / BVB, j = blockIdx.x % BVB;
    if (st[s].status != CG_RUNNING) return;
    const BatchSlice &d = sl[s];
    double a = 0.0;
    for (int i = threadIdx.x; i < d.nrow; i += blockDim.x) a += rpart[d.rpart + i];
    const double pAp = bsum(a);
    if (!(pAp > 0.0) || !(pAp < INFINITY)) {
        if (j == 0 && threadIdx.x == 0) st[s].status = CG_BREAKDOWN;
        return;
    }
    const double alpha = st[s].rr / pAp;
    const T al = (T)alpha;
    const size_t n = (size_t)d.N * d.N;
    double rr = 0.0;
    for (size_t i = (size_t)j * blockDim.x + threadIdx.x; i < n; i += (size_t)BVB * blockDim.x) {
        const size_t g = d.img + i;
        x[g] += al * p[g];
        const T ri = r[g] - al * Ap[g];
        r[g] = ri;
        rr += (double)ri * (double)ri;
    }
    rr = bsum(rr);
    if (threadIdx.x == 0) upart[blockIdx.x] = rr;
}

__global__ void __launch_bounds__(256) kb_cg_beta(CGState *st, const double *upart)
{
    const int s = blockIdx.x;
    if (st[s].status != CG_RUNNING) return;
    const double v = threadIdx.x < BVB ? upart[s * BVB + threadIdx.x] : 0.0;
    const double rr = bsum(v);
    if (threadIdx.x == 0) {
        CGState &c = st[s];
        const int64_t k = c.k + 1;
        c.k = k;
        c.ring[k % CG_RING] = rr;
        c.beta = rr / c.rr;
        c.rr = rr;
        if (!(rr == rr)) c.status = CG_BREAKDOWN;
        else if (rr <= c.thr2) c.status = CG_CONVERGED;
    }
}

// Residual replacement: a slice whose recursive residual met the rule while
// the recomputed one (st.pad, from A x in Ax) did not restarts from its
// iterate with r = b - A x, p = r; the iteration count continues.  Other
// slices keep their state.  Both kernels test the same condition on the
// same state.
__device__ __forceinline__ bool slice_restarts(const CGState &c)
{
    return c.status == CG_CONVERGED && c.pad > c.thr2;
}

template <typename T>
__global__ void __launch_bounds__(256)
kb_cg_restart_vec(const CGState *st, const BatchSlice *__restrict__ sl, const T *__restrict__ b,
                  const T *__restrict__ Ax, T *__restrict__ r, T *__restrict__ p, double *__restrict__ prr)
{
    const int s = blockIdx.x / BVB, j = blockIdx.x % BVB;
    if (!slice_restarts(st[s])) {
        if (threadIdx.x == 0) prr[blockIdx.x] = 0.0;
        return;
    }
    const BatchSlice &d = sl[s];
    const size_t n = (size_t)d.N * d.N;
    double rr = 0.0;
    for (size_t i = (size_t)j * blockDim.x + threadIdx.x; i < n; i += (size_t)BVB * blockDim.x) {
        const size_t g = d.img + i;
        const T ri = b[g] - Ax[g];
        r[g] = ri;
        p[g] = ri;
        rr += (double)ri * (double)ri;
    }
    rr = bsum(rr);
    if (threadIdx.x == 0) prr[blockIdx.x] = rr;
}

__global__ void __launch_bounds__(256) kb_cg_restart_fin(CGState *st, const double *prr)
{
    const int s = blockIdx.x;
    const bool go = slice_restarts(st[s]);
    const double rr = bsum(threadIdx.x < BVB ? prr[s * BVB + threadIdx.x] : 0.0);
    if (go && threadIdx.x == 0) {
        CGState &c = st[s];
        c.rr = rr;
        c.beta = 0.0;
        c.ring[c.k % CG_RING] = rr;
        c.status = (rr <= c.thr2) ? CG_CONVERGED : CG_RUNNING;
        if (!(rr == rr)) c.status = CG_BREAKDOWN;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
kb_resid(const BatchSlice *__restrict__ sl, const T *__restrict__ b, const T *__restrict__ Ax,
         double *__restrict__ part)
{
    const int s = blockIdx.x / BVB, j = blockIdx.x % BVB;
    const BatchSlice &d = sl[s];
    const size_t n = (size_t)d.N * d.N;
    double acc = 0.0;
    for (size_t i = (size_t)j * blockDim.x + threadIdx.x; i < n; i += (size_t)BVB * blockDim.x) {
        const double e = (double)b[d.img + i] - (double)Ax[d.img + i];
        acc += e * e;
    }
    acc = bsum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256) kb_resid_fin(CGState *st, const double *part)
{
    const int s = blockIdx.x;
    const double v = threadIdx.x < BVB ? part[s * BVB + threadIdx.x] : 0.0;
    const double r = bsum(v);
    if (threadIdx.x == 0) st[s].pad = r;
}

// ---------------------------------------------------------------------------
// Dispatch on (size code, E).  E candidates: fft_elems(P) and, for P = 2^k
// >= 512, fft_elems(P) / 2 (except P = 4096, which needs 16 at 256
// threads); for P = 3 * 2^k (1536, 3072), 24 and 12.
// ---------------------------------------------------------------------------
static bool e_ok(int pc, int E)
{
    const int P = fft_size(pc), E0 = fft_elems(P);
    if (E == E0) return true;
    if (P % 3 == 0) return (E == 12 || E == 24) && P / E <= 256;
    return P >= 512 && P <= 2048 && E == E0 / 2;
}

#define GCT_BCASE(kern, T, LG, E, grid, lds, s, ...) \
    hipLaunchKernelGGL((kern<T, LG, E>), grid, dim3(fft_size(LG) / E), lds, s, __VA_ARGS__)

#define GCT_LAUNCH_B(kern, T, pc, E, grid, lds, s, ...)                                         \
    do {                                                                                         \
        switch (pc) {                                                                          \
        case 2: GCT_BCASE(kern, T, 2, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 3: GCT_BCASE(kern, T, 3, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 4: GCT_BCASE(kern, T, 4, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 5: GCT_BCASE(kern, T, 5, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 6: GCT_BCASE(kern, T, 6, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 7: GCT_BCASE(kern, T, 7, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 8: GCT_BCASE(kern, T, 8, 4, grid, lds, s, __VA_ARGS__); break;                      \
        case 9:                                                                                  \
            if (E == 8) GCT_BCASE(kern, T, 9, 8, grid, lds, s, __VA_ARGS__);                     \
            else GCT_BCASE(kern, T, 9, 4, grid, lds, s, __VA_ARGS__);                            \
            break;                                                                               \
        case 10:                                                                                 \
            if (E == 16) GCT_BCASE(kern, T, 10, 16, grid, lds, s, __VA_ARGS__);                  \
            else GCT_BCASE(kern, T, 10, 8, grid, lds, s, __VA_ARGS__);                           \
            break;                                                                               \
        case 11:                                                                                 \
            if (E == 16) GCT_BCASE(kern, T, 11, 16, grid, lds, s, __VA_ARGS__);                  \
            else GCT_BCASE(kern, T, 11, 8, grid, lds, s, __VA_ARGS__);                           \
            break;                                                                               \
        case 12: GCT_BCASE(kern, T, 12, 16, grid, lds, s, __VA_ARGS__); break;                   \
        GCT_MIXED_CASES(GCT_BCASE, kern, T, E, grid, lds, s, __VA_ARGS__)                        \
        }                                                                                        \
    } while (0)

}  // namespace gct

using namespace gct;

// ---------------------------------------------------------------------------
// Host batch object
// ---------------------------------------------------------------------------
struct BatchGroup {
    int pc;
    int E[2];   // tuned elements per thread of the row passes, [f32, f64]
    int Ec[2];  // and of the column pass
    int2 *rows = nullptr, *cols = nullptr, *srows = nullptr, *scols = nullptr;
    int nrows = 0, ncols = 0, nsrows = 0, nscols = 0;
    // two row pairs per block (FP32 row passes of 1024- and 2048-point
    // groups whose slices all have even N): map of (slice, row quad)
    int2 *rows2 = nullptr;
    int nrows2 = 0;
};

// LDS of the two-pair row kernels
template <typename T>
inline size_t rows2_lds_bytes(int P, bool inv)
{
    const size_t data = inv ? 2 * (size_t)(P + 2) : 2 * (size_t)P;
    size_t b = (data + (twiddles_in_lds<T>(P) ? (size_t)(P / 2) : 0)) * sizeof(C2<T>);
    return b > 512 * sizeof(double) ? b : 512 * sizeof(double);
}

#define GCT_LAUNCH_B2(kern, T, pc, E, grid, lds, s, ...)                                               \
    do {                                                                                                \
        if (pc == 10 && E == 16) hipLaunchKernelGGL((kern<T, 10, 16>), grid, dim3(128), lds, s, __VA_ARGS__); \
        else if (pc == 10) hipLaunchKernelGGL((kern<T, 10, 8>), grid, dim3(256), lds, s, __VA_ARGS__);    \
        else if (E == 16) hipLaunchKernelGGL((kern<T, 11, 16>), grid, dim3(256), lds, s, __VA_ARGS__);      \
        else hipLaunchKernelGGL((kern<T, 11, 8>), grid, dim3(512), lds, s, __VA_ARGS__);                    \
    } while (0)

struct gct_batch {
    std::vector<const gct_plan *> plans;
    int S = 0;
    BatchSlice *dev[2] = {nullptr, nullptr};  // descriptors with f32 / f64 tables
    std::vector<BatchSlice> host;             // (f32 variant)
    int64_t img_total = 0, gram_total = 0, spec_total = 0, w_total = 0, rpart_total = 0;
    std::vector<BatchGroup> groups;
    int2 *gram_map = nullptr;
    int ngram = 0;
    std::vector<CGGraph> graphs;
    hipStream_t capture_stream = nullptr;
    int64_t dev_bytes = 0;  // bytes of the block maps and slice descriptors
    // Concurrent transform groups: the apply passes of the costliest group
    // run on the caller's stream, those of the others on `side`, forked and
    // joined through events (each group's three passes touch only its own
    // slices, so the chains are independent).
    int main_group = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

int upload_map(int2 **dst, const std::vector<int2> &v, int64_t *bytes)
{
    if (v.empty()) return GCT_OK;
    *bytes += (int64_t)(v.size() * sizeof(int2));
    hipError_t e = hipMalloc(dst, v.size() * sizeof(int2));
    if (e != hipSuccess) return check_hip(e, "hipMalloc(batch map)");
    return check_hip(hipMemcpy(*dst, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice),
                     "hipMemcpy(batch map)");
}

void free_batch(gct_batch *b)
{
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    for (auto &g : b->groups) {
        for (int2 *m : {g.rows, g.cols, g.srows, g.scols, g.rows2})
            if (m) (void)hipFree(m);
    }
    if (b->gram_map) (void)hipFree(b->gram_map);
    for (int i = 0; i < 2; ++i)
        if (b->dev[i]) (void)hipFree(b->dev[i]);
    delete b;
}

// workspace layout for the batched operations
struct BLayout {
    size_t W1, W2, R, r, p, Ap, rpart, upart, upart2, st, total;
};

BLayout blayout(const gct_batch *b, size_t elem)
{
    BLayout L{};
    size_t o = 0;
    L.W1 = o; o += align256((size_t)b->w_total * 2 * elem);
    L.W2 = o; o += align256((size_t)b->w_total * 2 * elem);
    L.R = L.W1;  // the spectrum scratch ((P/2+1) P complex per slice) reuses the start
    const size_t spec_scratch = align256((size_t)b->spec_total * 2 * elem);
    size_t apply_end = o;
    size_t cg_base = std::max(apply_end, spec_scratch);
    o = cg_base;
    L.r = o; o += align256((size_t)b->img_total * elem);
    L.p = o; o += align256((size_t)b->img_total * elem);
    L.Ap = o; o += align256((size_t)b->img_total * elem);
    L.rpart = o; o += align256((size_t)b->rpart_total * sizeof(double));
    L.upart = o; o += align256((size_t)b->S * BVB * sizeof(double));
    L.upart2 = o; o += align256((size_t)b->S * BVB * sizeof(double));
    L.st = o; o += align256((size_t)b->S * sizeof(CGState));
    L.total = o;
    return L;
}

template <typename T>
int dti() { return sizeof(T) == 4 ? 0 : 1; }

// The side stream and its events (default priority; made with the batch).
hipError_t batch_side(const gct_batch *b)
{
    gct_batch *mb = const_cast<gct_batch *>(b);
    hipError_t e = hipSuccess;
    if (!mb->side) e = hipStreamCreateWithFlags(&mb->side, hipStreamNonBlocking);
    if (e == hipSuccess && !mb->ev_fork) e = hipEventCreateWithFlags(&mb->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess && !mb->ev_join) e = hipEventCreateWithFlags(&mb->ev_join, hipEventDisableTiming);
    return e;
}

// The three passes of one transform group on stream s.
template <typename T>
void group_passes(const gct_batch *b, const BatchGroup &g, const T *Ghat, const T *src, T *y, C2<T> *W1, C2<T> *W2,
                  hipStream_t s, const CGState *st, T *pupd, const T *dotv, double *partial)
{
    const BatchSlice *sl = b->dev[dti<T>()];
    const int E = g.E[dti<T>()], Ec = g.Ec[dti<T>()];
    const size_t lds = fft_lds_bytes<T>(fft_size(g.pc), E), ldsc = fft_lds_bytes<T>(fft_size(g.pc), Ec);
    auto rows_fwd = [&]() {
        if constexpr (sizeof(T) == 4) {
            if (g.nrows2) {
                GCT_LAUNCH_B2(kb_rows_fwd2, T, g.pc, E, dim3(g.nrows2), rows2_lds_bytes<T>(fft_size(g.pc), false), s,
                              g.rows2, sl, src, W1, st, pupd);
                return;
            }
        }
        GCT_LAUNCH_B(kb_rows_fwd, T, g.pc, E, dim3(g.nrows), lds, s, g.rows, sl, src, W1, st, pupd);
    };
    auto rows_inv = [&]() {
        if constexpr (sizeof(T) == 4) {
            if (g.nrows2) {
                GCT_LAUNCH_B2(kb_rows_inv2, T, g.pc, E, dim3(g.nrows2), rows2_lds_bytes<T>(fft_size(g.pc), true), s,
                              g.rows2, sl, W2, y, st, dotv, partial);
                return;
            }
        }
        GCT_LAUNCH_B(kb_rows_inv, T, g.pc, E, dim3(g.nrows), lds, s, g.rows, sl, W2, y, st, dotv, partial);
    };
    rows_fwd();
    GCT_LAUNCH_B(kb_cols, T, g.pc, Ec, dim3(g.ncols), ldsc, s, g.cols, sl, W1, W2, Ghat, st);
    rows_inv();
}

template <typename T>
hipError_t batch_apply_passes(const gct_batch *b, const T *Ghat, const T *src, T *y, void *ws,
                              hipStream_t s, const CGState *st, T *pupd, const T *dotv,
                              double *partial)
{
    const BLayout L = blayout(b, sizeof(T));
    char *w = reinterpret_cast<char *>(ws);
    C2<T> *W1 = reinterpret_cast<C2<T> *>(w + L.W1), *W2 = reinterpret_cast<C2<T> *>(w + L.W2);
    const int ng = (int)b->groups.size();
    if (ng == 1) {
        group_passes<T>(b, b->groups[0], Ghat, src, y, W1, W2, s, st, pupd, dotv, partial);
        return hipGetLastError();
    }
    if (!b->side || !b->ev_fork || !b->ev_join) return hipErrorInvalidResourceHandle;
    hipError_t e = hipEventRecord(b->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
    if (e != hipSuccess) return e;
    for (int i = 0; i < ng; ++i)
        if (i != b->main_group) group_passes<T>(b, b->groups[i], Ghat, src, y, W1, W2, b->side, st, pupd, dotv, partial);
    group_passes<T>(b, b->groups[b->main_group], Ghat, src, y, W1, W2, s, st, pupd, dotv, partial);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join, 0);
    return e;
}

template <typename T>
hipError_t batch_spectrum(const gct_batch *b, const T *G, T *Ghat, void *ws, hipStream_t s)
{
    const BLayout L = blayout(b, sizeof(T));
    C2<T> *R = reinterpret_cast<C2<T> *>(reinterpret_cast<char *>(ws) + L.R);
    const BatchSlice *sl = b->dev[dti<T>()];
    for (const auto &g : b->groups) {
        const int E = g.E[dti<T>()];
        const size_t lds = fft_lds_bytes<T>(fft_size(g.pc), E);
        GCT_LAUNCH_B(kb_spec_rows, T, g.pc, E, dim3(g.nsrows), lds, s, g.srows, sl, G, R);
    }
    for (const auto &g : b->groups) {
        const int E = g.E[dti<T>()];
        const size_t lds = fft_lds_bytes<T>(fft_size(g.pc), E);
        GCT_LAUNCH_B(kb_spec_cols, T, g.pc, E, dim3(g.nscols), lds, s, g.scols, sl, R, Ghat);
    }
    return hipGetLastError();
}

#define B_TRY(call)                                          \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return check_hip(e_, #call);   \
    } while (0)

template <typename T>
int batch_cg(const gct_batch *b, const T *Ghat, const T *bv, T *x, int use_x0, double rtol, int max_iter,
             int check_every, gct_cg_result *res, void *ws, hipStream_t s)
{
    const BLayout L = blayout(b, sizeof(T));
    char *w = reinterpret_cast<char *>(ws);
    T *r = reinterpret_cast<T *>(w + L.r), *p = reinterpret_cast<T *>(w + L.p);
    T *Ap = reinterpret_cast<T *>(w + L.Ap);
    double *rpart = reinterpret_cast<double *>(w + L.rpart);
    double *upart = reinterpret_cast<double *>(w + L.upart);
    double *upart2 = reinterpret_cast<double *>(w + L.upart2);
    CGState *st = reinterpret_cast<CGState *>(w + L.st);
    const BatchSlice *sl = b->dev[dti<T>()];
    const int S = b->S;
    if (check_every <= 0) check_every = 8;
    if (use_x0) B_TRY(batch_apply_passes<T>(b, Ghat, x, Ap, ws, s, nullptr, nullptr, nullptr, nullptr));
    hipLaunchKernelGGL(kb_cg_init<T>, dim3(S * BVB), dim3(256), 0, s, sl, bv, x, r, p,
                       use_x0 ? (const T *)Ap : nullptr, upart, upart2);
    hipLaunchKernelGGL(kb_cg_init_fin, dim3(S), dim3(256), 0, s, st, (const double *)upart,
                       (const double *)upart2, rtol * rtol, use_x0);
    if (use_x0) hipLaunchKernelGGL(kb_cg_fallback_vec<T>, dim3(S * BVB), dim3(256), 0, s, (const CGState *)st, sl, bv, x, r, p);
    B_TRY(hipGetLastError());
    std::vector<CGState> hs(S);
    auto pull = [&]() -> int {
        B_TRY(hipMemcpyAsync(hs.data(), st, S * sizeof(CGState), hipMemcpyDeviceToHost, s));
        B_TRY(hipStreamSynchronize(s));
        return GCT_OK;
    };
    auto running = [&]() {
        for (const auto &c : hs)
            if (c.status == CG_RUNNING) return true;
        return false;
    };
    int rc = pull();
    if (rc) return rc;
    auto launch_iters = [&](int count, hipStream_t st_) -> hipError_t {
        for (int i = 0; i < count; ++i) {
            hipError_t e = batch_apply_passes<T>(b, Ghat, r, Ap, ws, st_, st, p, p, rpart);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kb_cg_update<T>, dim3(S * BVB), dim3(256), 0, st_, st, sl, x, r, p,
                               Ap, rpart, upart);
            hipLaunchKernelGGL(kb_cg_beta, dim3(S), dim3(256), 0, st_, st, upart);
        }
        return hipGetLastError();
    };
    // Runs: the first from the start vectors; later ones restart the slices
    // whose recursive residual met the rule while the recomputed one did not
    // (at most BATCH_MAX_RESTARTS, within max_iter iterations per slice).
    int64_t limit = max_iter;
    for (int run = 0;; ++run) {
        int64_t done = 0;
        while (running() && done < limit) {
            const int chunk = (int)std::min<int64_t>(check_every, limit - done);
            if (chunk == check_every) {
                const CGGraphKey key{(const void *)Ghat, (void *)x, ws, (int)sizeof(T), chunk};
                hipGraphExec_t exec = nullptr;
                for (const auto &g : b->graphs)
                    if (g.key == key) exec = g.exec;
                if (!exec) {
                    gct_batch *mb = const_cast<gct_batch *>(b);
                    if (!mb->capture_stream &&
                        hipStreamCreateWithFlags(&mb->capture_stream, hipStreamNonBlocking) != hipSuccess)
                        return fail(GCT_EHIP, "cannot create the capture stream");
                    B_TRY(hipStreamBeginCapture(mb->capture_stream, hipStreamCaptureModeThreadLocal));
                    hipError_t e = launch_iters(chunk, mb->capture_stream);
                    hipGraph_t gr = nullptr;
                    hipError_t e2 = hipStreamEndCapture(mb->capture_stream, &gr);
                    if (e != hipSuccess || e2 != hipSuccess) {
                        if (gr) (void)hipGraphDestroy(gr);
                        return check_hip(e != hipSuccess ? e : e2, "batch cg graph capture");
                    }
                    e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    if (e != hipSuccess) return check_hip(e, "hipGraphInstantiate");
                    if (mb->graphs.size() >= 8) {
                        (void)hipGraphExecDestroy(mb->graphs.front().exec);
                        mb->graphs.erase(mb->graphs.begin());
                    }
                    mb->graphs.push_back({key, exec});
                }
                B_TRY(hipGraphLaunch(exec, s));
            } else {
                B_TRY(launch_iters(chunk, s));
            }
            if ((rc = pull())) return rc;
            done += chunk;
        }
        // true residuals of the returned iterates (A x left in Ap)
        B_TRY(batch_apply_passes<T>(b, Ghat, x, Ap, ws, s, nullptr, nullptr, nullptr, nullptr));
        hipLaunchKernelGGL(kb_resid<T>, dim3(S * BVB), dim3(256), 0, s, sl, bv, Ap, upart);
        hipLaunchKernelGGL(kb_resid_fin, dim3(S), dim3(256), 0, s, st, upart);
        B_TRY(hipGetLastError());
        if ((rc = pull())) return rc;
        int64_t kmax = -1;
        for (const auto &c : hs)
            if (c.status == CG_CONVERGED && c.pad > c.thr2) kmax = std::max<int64_t>(kmax, c.k);
        if (kmax < 0 || run == BATCH_MAX_RESTARTS || kmax >= max_iter || running()) break;
        hipLaunchKernelGGL(kb_cg_restart_vec<T>, dim3(S * BVB), dim3(256), 0, s, (const CGState *)st, sl, bv,
                           (const T *)Ap, r, p, upart);
        hipLaunchKernelGGL(kb_cg_restart_fin, dim3(S), dim3(256), 0, s, st, (const double *)upart);
        B_TRY(hipGetLastError());
        if ((rc = pull())) return rc;
        limit = max_iter - kmax;
    }
    int worst = GCT_OK;
    for (int i = 0; i < S; ++i) {
        const CGState &c = hs[i];
        auto rel = [&](double v) { return c.bb > 0.0 ? std::sqrt(v / c.bb) : 0.0; };
        gct_cg_result &o = res[i];
        o.iters = (int32_t)c.k;
        o.rel_res = rel(c.rr);
        o.rel_res_true = rel(c.pad);
        o.rel_res0 = rel(c.rr0);
        o.fell_back = (int32_t)c.fb;
        // success means the recomputed residual met the rule too
        o.status = c.status == CG_CONVERGED ? (c.pad <= c.thr2 ? GCT_OK : GCT_ENOTCONV)
                   : c.status == CG_BREAKDOWN ? GCT_EBREAKDOWN
                                              : GCT_ENOTCONV;
        if (o.status == GCT_EBREAKDOWN) worst = GCT_EBREAKDOWN;
        else if (o.status == GCT_ENOTCONV && worst == GCT_OK) worst = GCT_ENOTCONV;
    }
    return worst;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int gct_batch_create(const gct_plan *const *plans, int32_t count, gct_batch **out)
{
    if (!out) return fail(GCT_EINVAL, "batch output pointer is NULL");
    *out = nullptr;
    if (!plans || count < 1) return fail(GCT_EINVAL, "need at least one plan");
    for (int i = 0; i < count; ++i)
        if (!plans[i]) return fail(GCT_EINVAL, "NULL plan in batch");
    gct_batch *b = new gct_batch();
    b->plans.assign(plans, plans + count);
    b->S = count;
    std::map<int, std::vector<int>> by_p;
    b->host.resize(count);
    for (int i = 0; i < count; ++i) {
        const gct_plan *p = plans[i];
        BatchSlice d{};
        d.N = p->N;
        d.pc = p->pc;
        d.n = p->gram_n;  // Gram-filter table entries
        d.nrow = (p->N + 1) / 2;
        d.img = b->img_total;
        b->img_total += (int64_t)p->N * p->N;
        d.gram = b->gram_total;
        b->gram_total += (int64_t)(2 * p->N - 1) * (2 * p->N - 1);
        d.spec = b->spec_total;
        b->spec_total += (int64_t)(p->P / 2 + 1) * p->P;
        d.w = b->w_total;
        b->w_total += (int64_t)(p->P / 2 + 1) * p->N;
        d.rpart = b->rpart_total;
        b->rpart_total += d.nrow;
        b->host[i] = d;
        by_p[p->pc].push_back(i);
    }
    // descriptors with the f32 and f64 tables of each plan
    for (int t = 0; t < 2; ++t) {
        std::vector<BatchSlice> v = b->host;
        for (int i = 0; i < count; ++i) {
            v[i].ga = t == 0 ? plans[i]->dev.gram_f32 : plans[i]->dev.gram_f64;
            v[i].gord = reinterpret_cast<const int32_t *>(plans[i]->dev.gram_ord);
            v[i].gth = reinterpret_cast<const double *>(plans[i]->dev.gram_th);
            v[i].ghmax = plans[i]->gram_hmax;
            v[i].l1 = plans[i]->lx1;
            v[i].l2 = plans[i]->lx2;
            v[i].gd4 = plans[i]->gram_d4;
            v[i].tw = t == 0 ? plans[i]->dev.tw_f32 : plans[i]->dev.tw_f64;
        }
        b->dev_bytes += (int64_t)(count * sizeof(BatchSlice));
        hipError_t e = hipMalloc(&b->dev[t], count * sizeof(BatchSlice));
        if (e == hipSuccess)
            e = hipMemcpy(b->dev[t], v.data(), count * sizeof(BatchSlice), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_batch(b);
            return check_hip(e, "batch descriptors");
        }
    }
    // block maps per FFT size
    for (auto &kv : by_p) {
        BatchGroup g;
        g.pc = kv.first;
        const int P = fft_size(g.pc);
        g.E[0] = g.E[1] = g.Ec[0] = g.Ec[1] = fft_elems(P);
        std::vector<int2> rows, cols, srows, scols, rows2;
        bool pair2 = g.pc == 10 || g.pc == 11;
        for (int i : kv.second) {
            const int N = plans[i]->N;
            pair2 = pair2 && N % 2 == 0 && b->host[i].w % 2 == 0;
            for (int k = 0; k < (N / 2 + 1) / 2; ++k) rows2.push_back(make_int2(i, k));
            for (int k = 0; k < (N + 1) / 2; ++k) rows.push_back(make_int2(i, k));
            for (int k = 0; k <= P / 2; ++k) cols.push_back(make_int2(i, k));
            for (int k = 0; k < P / 2; ++k) srows.push_back(make_int2(i, k));
            for (int k = 0; k <= P / 2; ++k) scols.push_back(make_int2(i, k));
        }
        g.nrows = (int)rows.size();
        g.ncols = (int)cols.size();
        g.nsrows = (int)srows.size();
        g.nscols = (int)scols.size();
        int rc = GCT_OK;
        if (!rc) rc = upload_map(&g.rows, rows, &b->dev_bytes);
        if (!rc) rc = upload_map(&g.cols, cols, &b->dev_bytes);
        if (!rc) rc = upload_map(&g.srows, srows, &b->dev_bytes);
        if (!rc) rc = upload_map(&g.scols, scols, &b->dev_bytes);
        if (!rc && pair2) {
            g.nrows2 = (int)rows2.size();
            rc = upload_map(&g.rows2, rows2, &b->dev_bytes);
        }
        b->groups.push_back(g);
        if (rc) {
            free_batch(b);
            return rc;
        }
    }
    // the costliest transform group (slices x P^2 log2 P) runs on the caller's stream
    {
        double best = -1.0;
        for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
            const double P = (double)fft_size(b->groups[gi].pc);
            const double cost = (double)b->groups[gi].ncols / (P / 2 + 1) * P * P * std::log2(P);
            if (cost > best) {
                best = cost;
                b->main_group = gi;
            }
        }
    }
    if (b->groups.size() > 1) {  // side stream and events made here, never during a capture
        const hipError_t e = batch_side(b);
        if (e != hipSuccess) {
            free_batch(b);
            return check_hip(e, "batch side stream");
        }
    }
    std::vector<int2> gm;
    for (int i = 0; i < count; ++i) {
        const int N = plans[i]->N, T = (N + GRAM_TILE - 1) / GRAM_TILE;
        // the tiles of the half plane k2 >= 0, or (eight symmetries) of the
        // octant 0 <= k2 <= k1
        const int tiles = plans[i]->gram_d4 ? T * (T + 1) / 2 : ((2 * N - 1 + GRAM_TILE - 1) / GRAM_TILE) * T;
        for (int k = 0; k < tiles; ++k) gm.push_back(make_int2(i, k));
    }
    b->ngram = (int)gm.size();
    int rc = upload_map(&b->gram_map, gm, &b->dev_bytes);
    if (rc) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return GCT_OK;
}

int gct_batch_device_bytes(const gct_batch *b, int64_t *bytes)
{
    if (!b || !bytes) return fail(GCT_EINVAL, "NULL argument");
    *bytes = b->dev_bytes;
    return GCT_OK;
}

int gct_batch_destroy(gct_batch *b)
{
    if (b) free_batch(b);
    return GCT_OK;
}

int gct_batch_get_info(const gct_batch *b, gct_batch_info *info, int64_t *image_offsets,
                       int64_t *gram_offsets, int64_t *spectrum_offsets)
{
    if (!b || !info) return fail(GCT_EINVAL, "NULL argument");
    info->slices = b->S;
    info->groups = (int32_t)b->groups.size();
    info->image_elems = b->img_total;
    info->gram_elems = b->gram_total;
    info->spectrum_elems = b->spec_total;
    for (int i = 0; i < b->S; ++i) {
        if (image_offsets) image_offsets[i] = b->host[i].img;
        if (gram_offsets) gram_offsets[i] = b->host[i].gram;
        if (spectrum_offsets) spectrum_offsets[i] = b->host[i].spec;
    }
    return GCT_OK;
}

size_t gct_batch_workspace_size(const gct_batch *b, int op, gct_dtype dt)
{
    if (!b) return 0;
    const BLayout L = blayout(b, dt == GCT_F64 ? 8 : 4);
    switch (op) {
    case GCT_OP_GRAM_SPECTRUM: return align256((size_t)b->spec_total * 2 * (dt == GCT_F64 ? 8 : 4));
    case GCT_OP_GRAM_APPLY: return L.W2 + align256((size_t)b->w_total * 2 * (dt == GCT_F64 ? 8 : 4));
    case GCT_OP_CG: return L.total;
    default: return 0;
    }
}

#define CHECK_BATCH_DT(b, dt)                                                         \
    do {                                                                              \
        if (!(b)) return fail(GCT_EINVAL, "batch is NULL");                           \
        if ((dt) != GCT_F32 && (dt) != GCT_F64) return fail(GCT_EINVAL, "bad dtype"); \
    } while (0)

int gct_batch_gram_build(const gct_batch *b, gct_dtype dt, void *G, void *stream)
{
    CHECK_BATCH_DT(b, dt);
    if (!G) return fail(GCT_EINVAL, "G is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32
                       ? launch_batch_gram_build<float>(b->gram_map, b->ngram, b->dev[0], (float *)G, s)
                       : launch_batch_gram_build<double>(b->gram_map, b->ngram, b->dev[1], (double *)G, s);
    return check_hip(e, "batch gram_build launch");
}

int gct_batch_gram_spectrum(const gct_batch *b, gct_dtype dt, const void *G, void *Ghat, void *ws,
                            void *stream)
{
    CHECK_BATCH_DT(b, dt);
    if (!G || !Ghat || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32 ? batch_spectrum<float>(b, (const float *)G, (float *)Ghat, ws, s)
                                 : batch_spectrum<double>(b, (const double *)G, (double *)Ghat, ws, s);
    return check_hip(e, "batch gram_spectrum launch");
}

int gct_batch_gram_apply(const gct_batch *b, gct_dtype dt, const void *Ghat, const void *c,
                         void *y, void *ws, void *stream)
{
    CHECK_BATCH_DT(b, dt);
    if (!Ghat || !c || !y || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (c == y) return fail(GCT_EINVAL, "y must not alias c");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32
                       ? batch_apply_passes<float>(b, (const float *)Ghat, (const float *)c, (float *)y,
                                                   ws, s, nullptr, nullptr, nullptr, nullptr)
                       : batch_apply_passes<double>(b, (const double *)Ghat, (const double *)c,
                                                    (double *)y, ws, s, nullptr, nullptr, nullptr,
                                                    nullptr);
    return check_hip(e, "batch gram_apply launch");
}

static int batch_cg_solve(const gct_batch *b, gct_dtype dt, const void *Ghat, const void *bv, void *x, int use_x0,
                          double rtol, int32_t max_iter, int32_t check_every, gct_cg_result *results,
                          void *ws, void *stream)
{
    CHECK_BATCH_DT(b, dt);
    if (!Ghat || !bv || !x || !ws || !results) return fail(GCT_EINVAL, "NULL argument");
    if (bv == x) return fail(GCT_EINVAL, "x must not alias b");
    if (max_iter < 0 || !(rtol >= 0.0)) return fail(GCT_EINVAL, "bad max_iter or rtol");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = dt == GCT_F32 ? batch_cg<float>(b, (const float *)Ghat, (const float *)bv, (float *)x, use_x0,
                                             rtol, max_iter, check_every, results, ws, s)
                           : batch_cg<double>(b, (const double *)Ghat, (const double *)bv,
                                              (double *)x, use_x0, rtol, max_iter, check_every, results, ws, s);
    if (rc == GCT_ENOTCONV) set_error("batch cg_solve: some slices reached max_iter");
    if (rc == GCT_EBREAKDOWN) set_error("batch cg_solve: breakdown in some slice");
    return rc;
}

int gct_batch_cg_solve(const gct_batch *b, gct_dtype dt, const void *Ghat, const void *bv, void *x,
                       double rtol, int32_t max_iter, int32_t check_every, gct_cg_result *results,
                       void *ws, void *stream)
{
    return batch_cg_solve(b, dt, Ghat, bv, x, 0, rtol, max_iter, check_every, results, ws, stream);
}

int gct_batch_cg_solve_x0(const gct_batch *b, gct_dtype dt, const void *Ghat, const void *bv, void *x,
                          double rtol, int32_t max_iter, int32_t check_every, gct_cg_result *results,
                          void *ws, void *stream)
{
    return batch_cg_solve(b, dt, Ghat, bv, x, 1, rtol, max_iter, check_every, results, ws, stream);
}

int gct_batch_get_pass_elems(const gct_batch *b, gct_dtype dt, int32_t *out)
{
    CHECK_BATCH_DT(b, dt);
    if (!out) return fail(GCT_EINVAL, "NULL output");
    const int t = dt == GCT_F32 ? 0 : 1;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        out[2 * gi] = b->groups[gi].E[t];
        out[2 * gi + 1] = b->groups[gi].Ec[t];
    }
    return GCT_OK;
}

int gct_batch_autotune(gct_batch *b, gct_dtype dt, const void *Ghat, void *ws, int32_t reps,
                       int32_t *chosen, void *stream)
{
    CHECK_BATCH_DT(b, dt);
    if (!Ghat || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    if (reps < 1) reps = 3;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int t = dt == GCT_F32 ? 0 : 1;
    const size_t elem = t == 0 ? 4 : 8;
    const BLayout L = blayout(b, elem);
    char *w = reinterpret_cast<char *>(ws);
    void *src = w + L.r, *dst = w + L.Ap;
    B_TRY(hipMemsetAsync(src, 0, (size_t)b->img_total * elem, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    // tune one group and one pass kind (row passes, then the column pass) at
    // a time, everything else keeping its current choice; each candidate is
    // timed on the whole batched apply.  On an error the pass keeps the
    // choice it had before its candidates were tried.
    for (int q = 0; q < 2 * (int)b->groups.size() && err == hipSuccess; ++q) {
        BatchGroup &g = b->groups[q / 2];
        int &Eq = q % 2 == 0 ? g.E[t] : g.Ec[t];
        const int P = fft_size(g.pc), E0 = fft_elems(P);
        const int before = Eq;
        int best = Eq;
        float best_ms = 1e30f;
        for (int E : {E0, E0 / 2}) {
            if (E < 4 || !e_ok(g.pc, E)) continue;
            Eq = E;
            for (int rep = 0; rep <= reps && err == hipSuccess; ++rep) {
                if (rep == 1) err = hipEventRecord(e0, s);
                if (err == hipSuccess)
                    err = t == 0 ? batch_apply_passes<float>(b, (const float *)Ghat, (const float *)src,
                                                             (float *)dst, ws, s, nullptr, nullptr, nullptr,
                                                             nullptr)
                                 : batch_apply_passes<double>(b, (const double *)Ghat, (const double *)src,
                                                              (double *)dst, ws, s, nullptr, nullptr, nullptr,
                                                              nullptr);
            }
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = E;
            }
        }
        Eq = err == hipSuccess ? best : before;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // captured CG graphs used the old shapes
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
    if (err != hipSuccess) return check_hip(err, "batch autotune");
    if (chosen)
        for (size_t gi = 0; gi < b->groups.size(); ++gi) chosen[gi] = b->groups[gi].E[t];
    return GCT_OK;
}

}  // extern "C"
