// Device bodies of the Gram-filtering passes (rows forward, columns,
// rows inverse) and of the spectrum passes, shared by the single-slice and
// the batched kernels.  Each body processes one transform with the P/E
// threads of its block; twiddles must be staged (stage_twiddles) and the
// block synchronised before the first body call.
#pragma once

#include "fft_common.h"
#include "gct_internal.h"

namespace gct {

// Logical index of block b of nb.  MI355X dispatches consecutive blocks
// round-robin over its 8 XCDs (block b on XCD b % 8), each with its own L2.
// The row passes read and write the transposed scratch arrays W1 / W2 a few
// bytes per cache line per row pair, so neighbouring row pairs must share
// an L2: this bijection gives each XCD a contiguous range of logical indices
// (the last nb % 8 blocks keep their own index).
__device__ __forceinline__ int xcd_swizzle(int b, int nb)
{
    constexpr int X = 8;
    const int q = nb / X;
    return b < q * X ? (b % X) * q + b / X : b;
}

// Twiddles go to LDS after the data area (fft_data_elems entries) when
// both fit in 64 KB, else they are read from the plan's global table.
template <typename T>
__host__ __device__ constexpr bool twiddles_in_lds(int P)
{
    return (size_t)(P + P / 2) * sizeof(C2<T>) <= 65536;
}

// HP twiddles by a block of NT threads (the launch's block size): every
// thread issues all its loads before its first LDS store, so the block
// waits for one global latency rather than one per round of NT entries.
template <typename T, bool TWL, int HP, int NT>
__device__ __forceinline__ const C2<T> *stage_twiddles(C2<T> *lds_after_data, const C2<T> *__restrict__ tw)
{
    if (!TWL) return tw;
    constexpr int K = (HP + NT - 1) / NT;
    C2<T> r[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int i = threadIdx.x + j * NT;
        if (HP % NT == 0 || i < HP) r[j] = tw[i];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int i = threadIdx.x + j * NT;
        if (HP % NT == 0 || i < HP) lds_after_data[i] = r[j];
    }
    return lds_after_data;
}

// Two adjacent complex values as one 16-byte access (FP32; the caller
// guarantees 16-byte alignment); FP64 falls back to two accesses.
template <typename T>
__device__ __forceinline__ void store_pair(C2<T> *p, const C2<T> &a, const C2<T> &b)
{
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(a.x, a.y, b.x, b.y);
    } else {
        p[0] = a;
        p[1] = b;
    }
}

template <typename T>
__device__ __forceinline__ void load_pair(const C2<T> *p, C2<T> &a, C2<T> &b)
{
    if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        a = {v.x, v.y};
        b = {v.z, v.w};
    } else {
        a = p[0];
        b = p[1];
    }
}

// Rows forward: real FFT of image rows ra and ra+1 (one complex transform),
// written transposed as W1[k][row], k in [0, P/2].  From registers: v[q]
// holds (row ra, row ra+1) at column t + G q (zero past N); one complex
// FFT, split into the two real-row spectra.
template <typename T, int PC, int E>
__device__ __forceinline__ void rows_fwd_regs(int ra, C2<T> (&v)[E], C2<T> *__restrict__ W1, int N, C2<T> *x,
                                              const C2<T> *tws)
{
    constexpr int P = fft_size(PC), hP = P >> 1, G = P / E;
    const int t = threadIdx.x;
    const int rb = ra + 1;
    fft_passes<T, E, P, 1, false, true>(v, x, t, tws);
    // split the two real rows: Xa = (Z[k] + conj Z[-k])/2, Xb = (Z[k] - conj Z[-k])/(2i)
#pragma unroll
    for (int q = 0; q < E; ++q) x[t + G * q] = v[q];
    __syncthreads();
    // rows ra, ra+1 of a column are adjacent in W1: one 16-byte store for
    // both (FP32) where they are 16-byte aligned (N even, aligned base)
    const bool pair = sizeof(T) == 4 && (N & 1) == 0 && (reinterpret_cast<uintptr_t>(W1) & 15) == 0;
    for (int k = t; k <= hP; k += G) {
        const C2<T> Zk = x[k], Zm = x[(P - k) % P];
        const C2<T> a = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        const C2<T> b = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
        if (pair) {
            store_pair(W1 + (size_t)k * N + ra, a, b);
        } else {
            W1[(size_t)k * N + ra] = a;
            if (rb < N) W1[(size_t)k * N + rb] = b;
        }
    }
    __syncthreads();  // x may be reused by the caller
}

// The load halves (rows_fwd_load, cols_load, rows_inv_load) touch no LDS
// and no twiddles, so a kernel can issue them before staging the twiddles:
// the two global latencies then overlap.  rows_fwd_load: with pupd, the
// rows are first updated in place as p = src + bt * p (CG direction
// update).
template <typename T, int PC, int E>
__device__ __forceinline__ void rows_fwd_load(int ra, const T *__restrict__ src, int N, T *pupd, T bt,
                                              C2<T> (&v)[E])
{
    constexpr int P = fft_size(PC), G = P / E;
    const int t = threadIdx.x;
    const bool hb = ra + 1 < N;  // row ra < N always
    const size_t oa = (size_t)ra * N, ob = hb ? oa + N : oa;
    // unconditional loads from clamped in-range addresses, masked afterwards:
    // no branch between them, so all are in flight before the first wait.
    // Entries q >= E/2 sit at t + G q >= P/2 >= N (P >= 2N): zero padding,
    // known at compile time, so the first transform pass drops their terms.
    constexpr int H = E / 2;
    T a[H], b[H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const int nc = min(t + G * q, N - 1);
        a[q] = src[oa + nc];
        b[q] = src[ob + nc];
    }
    if (pupd) {
        T ua[H], ub[H];
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const int nc = min(t + G * q, N - 1);
            ua[q] = pupd[oa + nc];
            ub[q] = pupd[ob + nc];
        }
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const int n = t + G * q;
            if (n >= N) continue;
            a[q] += bt * ua[q];
            pupd[oa + n] = a[q];
            if (hb) {
                b[q] += bt * ub[q];
                pupd[ob + n] = b[q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < E; ++q) {
        if (q >= H) {
            v[q] = {T(0), T(0)};
            continue;
        }
        const bool ok = t + G * q < N;
        v[q] = {ok ? a[q] : T(0), ok && hb ? b[q] : T(0)};
    }
}

template <typename T, int PC, int E>
__device__ __forceinline__ void body_rows_fwd(int ra, const T *__restrict__ src,
                                              C2<T> *__restrict__ W1, int N, C2<T> *x,
                                              const C2<T> *tws, T *pupd, T bt)
{
    C2<T> v[E];
    rows_fwd_load<T, PC, E>(ra, src, N, pupd, bt, v);
    rows_fwd_regs<T, PC, E>(ra, v, W1, N, x, tws);
}

// Columns: FFT along k2 of column col (N nonzero of P), times the real
// spectrum, inverse FFT (in registers between the two), first N entries.
template <typename T, int PC, int E>
__device__ __forceinline__ void cols_load(int col, const C2<T> *__restrict__ W1, const T *__restrict__ Ghat,
                                          int N, C2<T> (&v)[E], T (&gs)[E])
{
    constexpr int P = fft_size(PC), G = P / E;
    const int t = threadIdx.x;
    const C2<T> *in = W1 + (size_t)col * N;
    const T *g = Ghat + (size_t)col * P;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = t + G * q;
        // q >= E/2: n >= P/2 >= N, zero padding known at compile time
        v[q] = q < E / 2 && n < N ? in[n] : C2<T>{T(0), T(0)};
        gs[q] = g[n];
    }
}

template <typename T, int PC, int E>
__device__ __forceinline__ void cols_regs(int col, C2<T> (&v)[E], const T (&gs)[E], C2<T> *__restrict__ W2,
                                          int N, C2<T> *x, const C2<T> *tws)
{
    constexpr int P = fft_size(PC), G = P / E;
    const int t = threadIdx.x;
    fft_passes<T, E, P, 1, false, true>(v, x, t, tws);
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = {v[q].x * gs[q], v[q].y * gs[q]};
    fft_passes<T, E, P, 1, true, true>(v, x, t, tws);
    C2<T> *out = W2 + (size_t)col * N;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {  // n >= P/2 >= N for q >= E/2: the last pass drops them
        const int n = t + G * q;
        if (n < N) out[n] = v[q];
    }
}

// Rows inverse: Hermitian row spectra of rows ra, ra+1 (loaded as one
// complex spectrum) -> one complex inverse FFT (fft_passes) -> v[q] =
// (row ra, row ra+1) at column t + G q -> two real rows of y.
template <typename T, int PC, int E>
__device__ __forceinline__ void rows_inv_load(int ra, const C2<T> *__restrict__ W2, int N, C2<T> (&v)[E])
{
    constexpr int P = fft_size(PC), hP = P >> 1, G = P / E;
    const int t = threadIdx.x;
    const int rb = ra + 1;
    const bool pair = sizeof(T) == 4 && (N & 1) == 0 && (reinterpret_cast<uintptr_t>(W2) & 15) == 0;
    // one loop per access form, so that no load waits for the previous one
    C2<T> Ya[E], Yb[E];
    if (pair) {  // rows ra, ra+1 in one 16-byte load
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int k = t + G * q;
            const int kk = k <= hP ? k : P - k;  // Hermitian extension
            load_pair(W2 + (size_t)kk * N + ra, Ya[q], Yb[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int k = t + G * q;
            const int kk = k <= hP ? k : P - k;
            Ya[q] = W2[(size_t)kk * N + ra];
            Yb[q] = rb < N ? W2[(size_t)kk * N + rb] : C2<T>{T(0), T(0)};
        }
    }
#pragma unroll
    for (int q = 0; q < E; ++q) {
        if (t + G * q > hP) {
            Ya[q].y = -Ya[q].y;
            Yb[q].y = -Yb[q].y;
        }
        v[q] = {Ya[q].x - Yb[q].y, Ya[q].y + Yb[q].x};
    }
}

// The two real output rows from v (after the inverse transform) into y;
// returns this thread's FP64 partial of dotv . y (0 if dotv is null).
template <typename T, int PC, int E>
__device__ __forceinline__ double rows_inv_store(int ra, const C2<T> (&v)[E], T *__restrict__ y, int N,
                                                 const T *__restrict__ dotv)
{
    constexpr int P = fft_size(PC), G = P / E;
    const int t = threadIdx.x;
    const int rb = ra + 1;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {  // n >= P/2 >= N for q >= E/2
        const int n = t + G * q;
        if (n >= N) continue;
        y[(size_t)ra * N + n] = v[q].x;
        if (dotv) acc += (double)dotv[(size_t)ra * N + n] * (double)v[q].x;
        if (rb < N) {
            y[(size_t)rb * N + n] = v[q].y;
            if (dotv) acc += (double)dotv[(size_t)rb * N + n] * (double)v[q].y;
        }
    }
    return acc;
}

// Two block-wide FP64 sums at once: butterfly within each 64-lane wave,
// then the per-wave results (at most 4 waves) added in wave order through
// LDS (2 doubles per wave at red).  One barrier; the same order everywhere,
// so every block reducing the same data gets the same bits.
template <int NT>  // the block's thread count
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    constexpr int nw = (NT + 63) >> 6;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * wv] = a;
        red[2 * wv + 1] = b;
    }
    __syncthreads();
    a = red[0];
    b = red[1];
    for (int i = 1; i < nw; ++i) {
        a += red[2 * i];
        b += red[2 * i + 1];
    }
}

// Block-wide FP64 sum through an LDS area of blockDim doubles (all threads
// call it; the area is free again on return).
__device__ __forceinline__ double block_sum_lds(double v, double *red)
{
    __syncthreads();
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

// ---------------------------------------------------------------------------
// Spectrum of the circulant embedding of G.  Embedded position q in [0, P)
// holds tap q (q <= N-1) or q - P (q >= P-N+1); other positions are zero.
// ---------------------------------------------------------------------------
constexpr int NO_TAP = 1 << 30;
__device__ __forceinline__ int embed_tap(int q, int N, int P)
{
    if (q <= N - 1) return q;
    if (q >= P - N + 1) return q - P;
    return NO_TAP;
}

// embedded rows 2 seq and 2 seq + 1 -> R[k][row], k in [0, P/2]
template <typename T, int PC, int E>
__device__ __forceinline__ void body_spec_rows(int seq, const T *__restrict__ G,
                                               C2<T> *__restrict__ R, int N, C2<T> *x,
                                               const C2<T> *tws)
{
    constexpr int P = fft_size(PC), hP = P >> 1, Gt = P / E;
    const int t = threadIdx.x, W = 2 * N - 1;
    const int ka = embed_tap(2 * seq, N, P), kb = embed_tap(2 * seq + 1, N, P);
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int k1 = embed_tap(t + Gt * q, N, P);
        T re = 0, im = 0;
        if (k1 != NO_TAP) {
            if (ka != NO_TAP) re = G[(size_t)(ka + N - 1) * W + (k1 + N - 1)];
            if (kb != NO_TAP) im = G[(size_t)(kb + N - 1) * W + (k1 + N - 1)];
        }
        v[q] = {re, im};
    }
    fft_passes<T, E, P, 1, false, true>(v, x, t, tws);
#pragma unroll
    for (int q = 0; q < E; ++q) x[t + Gt * q] = v[q];
    __syncthreads();
    for (int k = t; k <= hP; k += Gt) {
        const C2<T> Zk = x[k], Zm = x[(P - k) % P];
        R[(size_t)k * P + 2 * seq] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        R[(size_t)k * P + 2 * seq + 1] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
    }
    __syncthreads();
}

// column k of R -> Ghat[k][.] = Re FFT / P^2
template <typename T, int PC, int E>
__device__ __forceinline__ void body_spec_cols(int col, const C2<T> *__restrict__ R,
                                               T *__restrict__ Ghat, C2<T> *x, const C2<T> *tws,
                                               T scale)
{
    constexpr int P = fft_size(PC), Gt = P / E;
    const int t = threadIdx.x;
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = R[(size_t)col * P + t + Gt * q];
    fft_passes<T, E, P, 1, false, true>(v, x, t, tws);
#pragma unroll
    for (int q = 0; q < E; ++q) Ghat[(size_t)col * P + t + Gt * q] = v[q].x * scale;
}

// LDS bytes of a pass kernel: data (P, or 2P with ping-pong) + twiddles
// (P/2, when in LDS), at least blockDim doubles for the reductions.
template <typename T>
inline size_t fft_lds_bytes(int P, int E)
{
    size_t b = (size_t)fft_data_elems<T>(P) * sizeof(C2<T>) +
               (twiddles_in_lds<T>(P) ? (size_t)(P / 2) * sizeof(C2<T>) : 0);
    const size_t red = (size_t)(P / E) * sizeof(double);
    return b > red ? b : red;
}

// Switch cases of the P = 3 * 2^k transforms (size codes 41 and 42: 1536
// and 3072 points) for a launch macro CASE(kern, T, code, E, grid, lds, s,
// ...), E = 24 or 12.
#define GCT_MIXED_CASES(CASE, kern, T, E, grid, lds, s, ...)                       \
    case 41:                                                                       \
        if (E == 12) CASE(kern, T, 41, 12, grid, lds, s, __VA_ARGS__);             \
        else CASE(kern, T, 41, 24, grid, lds, s, __VA_ARGS__);                     \
        break;                                                                     \
    default:                                                                       \
        if (E == 12) CASE(kern, T, 42, 12, grid, lds, s, __VA_ARGS__);             \
        else CASE(kern, T, 42, 24, grid, lds, s, __VA_ARGS__);                     \
        break;

// Valid (size code, E) pairs: E in {4, 8, 16} for powers of two, {12, 24}
// for three times a power of two; E divides P, at most 256 threads.
__host__ __device__ constexpr bool fft_combo_ok(int pc, int E)
{
    return ((pc >= 2 && pc <= 12 && (E == 4 || E == 8 || E == 16)) ||
            (pc >= 41 && pc <= 42 && (E == 12 || E == 24))) &&
           fft_size(pc) % E == 0 && (fft_size(pc) / E) <= 256;
}

}  // namespace gct
