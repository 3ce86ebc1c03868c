// Gram filtering (Sec. 4, closing remark): H^T H is Toeplitz-block-Toeplitz,
// so y = H^T H c is the zero-padded linear convolution of the N x N
// coefficients with the (2N-1)^2 Gram filter.  It is evaluated exactly (up
// to rounding) through the P x P circulant embedding, P >= 2N-1 a power of
// two: y = IFFT2(Ghat . FFT2(c_padded))[0:N, 0:N], with Ghat real and even
// because G[k] = G[-k].
//
// Three passes, each a group-local FFT in LDS (fft_common.h):
//   rows:    pairs of image rows -> one complex FFT -> two real-row spectra,
//            written transposed as W1[w1][k2], w1 in [0, P/2];
//   columns: per w1, FFT along k2 (N nonzero of P), times Ghat[w1][.],
//            inverse FFT, keep k2 < N -> W2[w1][k2];
//   rows:    pairs of Hermitian row spectra -> one complex inverse FFT ->
//            two real output rows, keep k1 < N.
// The 1/P^2 normalisation is folded into Ghat.  A group of P/4 threads owns
// one transform; a block holds nf groups (256 threads when P <= 1024).
#include <algorithm>

#include "fft_common.h"
#include "gct_internal.h"

namespace gct {

// Status word of a running CG solve (see cg.hip): kernels return at once
// when it is non-zero, so iterations queued after convergence cost only a
// launch.
__device__ __forceinline__ bool halted(const int64_t *status) { return status && *status != 0; }

// Twiddles: copied to LDS after the data area when TWL, else read from the
// plan's global table.
template <typename T, bool TWL>
__device__ __forceinline__ const C2<T> *stage_twiddles(C2<T> *lds_after_data,
                                                       const C2<T> *__restrict__ tw, int hP)
{
    if (!TWL) return tw;
    for (int i = threadIdx.x; i < hP; i += blockDim.x) lds_after_data[i] = tw[i];
    return lds_after_data;
}

// ---------------------------------------------------------------------------
// Pass 1: forward real FFT of image rows.  With `pupd` set (CG), the row
// vector is first updated in place as p = r + beta p (beta read from *beta).
// ---------------------------------------------------------------------------
template <typename T, bool TWL>
__global__ void __launch_bounds__(1024)
k_rows_fwd(const T *__restrict__ src, C2<T> *__restrict__ W1, int N, int logP, int nf,
           const C2<T> *__restrict__ tw, const int64_t *status, T *pupd, const double *beta)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = 1 << logP, Q = P >> 2, hP = P >> 1;
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, TWL>(buf + nf * P, tw, hP);
    const int f = threadIdx.x / Q, t = threadIdx.x - f * Q;
    const int seq = blockIdx.x * nf + f;
    const int ra = 2 * seq, rb = ra + 1;
    C2<T> *x = buf + f * P;
    const T bt = pupd ? (T)(*beta) : T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = t + q * Q;
        T re = 0, im = 0;
        if (n < N) {
            if (ra < N) {
                const size_t i = (size_t)ra * N + n;
                re = src[i];
                if (pupd) {
                    re += bt * pupd[i];
                    pupd[i] = re;
                }
            }
            if (rb < N) {
                const size_t i = (size_t)rb * N + n;
                im = src[i];
                if (pupd) {
                    im += bt * pupd[i];
                    pupd[i] = im;
                }
            }
        }
        x[n] = {re, im};
    }
    __syncthreads();
    fft_inplace<T, false>(x, logP, t, tws);
    // split the two real rows: Xa = (Z[k] + conj Z[-k])/2, Xb = (Z[k] - conj Z[-k])/(2i)
    for (int k = t; k <= hP; k += Q) {
        const C2<T> Zk = x[k], Zm = x[(P - k) & (P - 1)];
        if (ra < N) W1[(size_t)k * N + ra] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        if (rb < N) W1[(size_t)k * N + rb] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
    }
}

// ---------------------------------------------------------------------------
// Pass 2: per frequency column w1: FFT along k2, multiply by the real
// spectrum, inverse FFT, keep the first N entries.
// ---------------------------------------------------------------------------
template <typename T, bool TWL>
__global__ void __launch_bounds__(1024)
k_cols(const C2<T> *__restrict__ W1, C2<T> *__restrict__ W2, const T *__restrict__ Ghat, int N,
       int logP, int nf, const C2<T> *__restrict__ tw, const int64_t *status)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = 1 << logP, Q = P >> 2, hP = P >> 1;
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, TWL>(buf + nf * P, tw, hP);
    const int f = threadIdx.x / Q, t = threadIdx.x - f * Q;
    const int col = blockIdx.x * nf + f;
    const bool live = col <= hP;
    C2<T> *x = buf + f * P;
    const C2<T> *in = W1 + (size_t)col * N;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = t + q * Q;
        x[n] = (live && n < N) ? in[n] : C2<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_inplace<T, false>(x, logP, t, tws);
    const T *g = Ghat + (size_t)col * P;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = t + q * Q;
        const T s = live ? g[n] : T(0);
        x[n] = {x[n].x * s, x[n].y * s};
    }
    __syncthreads();
    fft_inplace<T, true>(x, logP, t, tws);
    if (live) {
        C2<T> *out = W2 + (size_t)col * N;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n = t + q * Q;
            if (n < N) out[n] = x[n];
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse real FFT of row spectra.  With `dotv` set (CG), each block
// also writes the FP64 partial sum of dotv . y over its rows.
// ---------------------------------------------------------------------------
template <typename T, bool TWL>
__global__ void __launch_bounds__(1024)
k_rows_inv(const C2<T> *__restrict__ W2, T *__restrict__ y, int N, int logP, int nf,
           const C2<T> *__restrict__ tw, const int64_t *status, const T *__restrict__ dotv,
           double *__restrict__ partial)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = 1 << logP, Q = P >> 2, hP = P >> 1;
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, TWL>(buf + nf * P, tw, hP);
    const int f = threadIdx.x / Q, t = threadIdx.x - f * Q;
    const int seq = blockIdx.x * nf + f;
    const int ra = 2 * seq, rb = ra + 1;
    C2<T> *x = buf + f * P;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = t + q * Q;
        C2<T> Ya = {T(0), T(0)}, Yb = {T(0), T(0)};
        const int kk = k <= hP ? k : P - k;  // Hermitian extension
        if (ra < N) Ya = W2[(size_t)kk * N + ra];
        if (rb < N) Yb = W2[(size_t)kk * N + rb];
        if (k > hP) {
            Ya.y = -Ya.y;
            Yb.y = -Yb.y;
        }
        x[k] = {Ya.x - Yb.y, Ya.y + Yb.x};
    }
    __syncthreads();
    fft_inplace<T, true>(x, logP, t, tws);
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = t + q * Q;
        if (n >= N) continue;
        const C2<T> v = x[n];
        if (ra < N) {
            y[(size_t)ra * N + n] = v.x;
            if (dotv) acc += (double)dotv[(size_t)ra * N + n] * (double)v.x;
        }
        if (rb < N) {
            y[(size_t)rb * N + n] = v.y;
            if (dotv) acc += (double)dotv[(size_t)rb * N + n] * (double)v.y;
        }
    }
    if (partial) {
        // reuse the LDS area (the launcher sizes it to >= blockDim doubles)
        __syncthreads();
        double *red = reinterpret_cast<double *>(smem_raw);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
    }
}

// ---------------------------------------------------------------------------
// Spectrum of the circulant embedding of G.
// ---------------------------------------------------------------------------
// Embedded tap index: position q in [0, P) holds tap q (q <= N-1) or
// q - P (q >= P-N+1); other positions are zero.
constexpr int NO_TAP = 1 << 30;
__device__ __forceinline__ int embed_tap(int q, int N, int P)
{
    if (q <= N - 1) return q;
    if (q >= P - N + 1) return q - P;
    return NO_TAP;
}

template <typename T, bool TWL>
__global__ void __launch_bounds__(1024)
k_spec_rows(const T *__restrict__ G, C2<T> *__restrict__ R, int N, int logP, int nf,
            const C2<T> *__restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = 1 << logP, Q = P >> 2, hP = P >> 1, W = 2 * N - 1;
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, TWL>(buf + nf * P, tw, hP);
    const int f = threadIdx.x / Q, t = threadIdx.x - f * Q;
    const int seq = blockIdx.x * nf + f;  // embedded row pair (2 seq, 2 seq + 1), < P/2
    const int ka = embed_tap(2 * seq, N, P), kb = embed_tap(2 * seq + 1, N, P);
    C2<T> *x = buf + f * P;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int q1 = t + q * Q;
        const int k1 = embed_tap(q1, N, P);
        T re = 0, im = 0;
        if (k1 != NO_TAP && seq < hP) {
            if (ka != NO_TAP) re = G[(size_t)(ka + N - 1) * W + (k1 + N - 1)];
            if (kb != NO_TAP) im = G[(size_t)(kb + N - 1) * W + (k1 + N - 1)];
        }
        x[q1] = {re, im};
    }
    __syncthreads();
    fft_inplace<T, false>(x, logP, t, tws);
    if (seq < hP) {
        for (int k = t; k <= hP; k += Q) {
            const C2<T> Zk = x[k], Zm = x[(P - k) & (P - 1)];
            R[(size_t)k * P + 2 * seq] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
            R[(size_t)k * P + 2 * seq + 1] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
        }
    }
}

template <typename T, bool TWL>
__global__ void __launch_bounds__(1024)
k_spec_cols(const C2<T> *__restrict__ R, T *__restrict__ Ghat, int logP, int nf,
            const C2<T> *__restrict__ tw, T scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = 1 << logP, Q = P >> 2, hP = P >> 1;
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, TWL>(buf + nf * P, tw, hP);
    const int f = threadIdx.x / Q, t = threadIdx.x - f * Q;
    const int col = blockIdx.x * nf + f;
    const bool live = col <= hP;
    C2<T> *x = buf + f * P;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = t + q * Q;
        x[n] = live ? R[(size_t)col * P + n] : C2<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_inplace<T, false>(x, logP, t, tws);
    if (live) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n = t + q * Q;
            Ghat[(size_t)col * P + n] = x[n].x * scale;
        }
    }
}

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
struct FftCfg {
    int Q;         // threads per transform (P/4)
    int nf;        // transforms per block
    int threads;   // nf * Q
    size_t lds;    // bytes of dynamic LDS
    bool twl;      // twiddles staged in LDS
};

template <typename T>
static FftCfg fft_cfg(int logP)
{
    FftCfg c;
    const int P = 1 << logP;
    c.Q = P >> 2;
    c.nf = c.Q >= 256 ? 1 : 256 / c.Q;
    c.threads = c.nf * c.Q;
    const size_t data = (size_t)c.nf * P * sizeof(C2<T>);
    const size_t twb = (size_t)(P / 2) * sizeof(C2<T>);
    c.twl = data + twb <= 65536;
    c.lds = data + (c.twl ? twb : 0);
    c.lds = std::max(c.lds, (size_t)c.threads * sizeof(double));
    return c;
}

template <typename T>
static const C2<T> *twiddles(const gct_plan *p)
{
    return reinterpret_cast<const C2<T> *>(sizeof(T) == 4 ? p->dev.tw_f32 : p->dev.tw_f64);
}

size_t apply_ws_bytes(const gct_plan *p, size_t elem)
{
    return 2 * align256((size_t)(p->P / 2 + 1) * p->N * 2 * elem);
}

size_t spectrum_ws_bytes(const gct_plan *p, size_t elem)
{
    return align256((size_t)(p->P / 2 + 1) * p->P * 2 * elem);
}

int apply_row_blocks(const gct_plan *p, size_t elem)
{
    const int nf = elem == 4 ? fft_cfg<float>(p->logP).nf : fft_cfg<double>(p->logP).nf;
    const int seqs = (p->N + 1) / 2;
    return (seqs + nf - 1) / nf;
}

#define GCT_LAUNCH_TWL(kern, T, twl, grid, block, lds, s, ...)                                  \
    do {                                                                                       \
        if (twl) hipLaunchKernelGGL((kern<T, true>), grid, block, lds, s, __VA_ARGS__);       \
        else hipLaunchKernelGGL((kern<T, false>), grid, block, lds, s, __VA_ARGS__);          \
    } while (0)

// The three passes of one apply; status/pupd/beta/dotv/partial are the CG
// hooks (all null for a plain apply).
template <typename T>
hipError_t launch_apply_passes(const gct_plan *p, const T *Ghat, const T *src, T *y, void *ws,
                               hipStream_t s, const int64_t *status, T *pupd, const double *beta,
                               const T *dotv, double *partial)
{
    const int N = p->N, P = p->P, logP = p->logP;
    const FftCfg c = fft_cfg<T>(logP);
    const size_t w1 = align256((size_t)(P / 2 + 1) * N * 2 * sizeof(T));
    C2<T> *W1 = reinterpret_cast<C2<T> *>(ws);
    C2<T> *W2 = reinterpret_cast<C2<T> *>(reinterpret_cast<char *>(ws) + w1);
    const C2<T> *tw = twiddles<T>(p);
    const int rblocks = apply_row_blocks(p, sizeof(T));
    const int cblocks = (P / 2 + 1 + c.nf - 1) / c.nf;
    GCT_LAUNCH_TWL(k_rows_fwd, T, c.twl, dim3(rblocks), dim3(c.threads), c.lds, s, src, W1, N, logP,
                   c.nf, tw, status, pupd, beta);
    GCT_LAUNCH_TWL(k_cols, T, c.twl, dim3(cblocks), dim3(c.threads), c.lds, s, W1, W2, Ghat, N, logP,
                   c.nf, tw, status);
    GCT_LAUNCH_TWL(k_rows_inv, T, c.twl, dim3(rblocks), dim3(c.threads), c.lds, s, W2, y, N, logP,
                   c.nf, tw, status, dotv, partial);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gram_apply(const gct_plan *p, const T *Ghat, const T *c, T *y, void *ws,
                             hipStream_t s)
{
    return launch_apply_passes<T>(p, Ghat, c, y, ws, s, nullptr, nullptr, nullptr, nullptr,
                                  nullptr);
}

template <typename T>
hipError_t launch_gram_spectrum(const gct_plan *p, const T *G, T *Ghat, void *ws, hipStream_t s)
{
    const int N = p->N, P = p->P, logP = p->logP;
    const FftCfg c = fft_cfg<T>(logP);
    C2<T> *R = reinterpret_cast<C2<T> *>(ws);
    const C2<T> *tw = twiddles<T>(p);
    const int rblocks = (P / 2 + c.nf - 1) / c.nf;  // P/2 embedded row pairs
    GCT_LAUNCH_TWL(k_spec_rows, T, c.twl, dim3(rblocks), dim3(c.threads), c.lds, s, G, R, N, logP,
                   c.nf, tw);
    const T scale = T(1.0 / ((double)P * (double)P));
    const int cblocks = (P / 2 + 1 + c.nf - 1) / c.nf;
    GCT_LAUNCH_TWL(k_spec_cols, T, c.twl, dim3(cblocks), dim3(c.threads), c.lds, s, R, Ghat, logP,
                   c.nf, tw, scale);
    return hipGetLastError();
}

template hipError_t launch_gram_apply<float>(const gct_plan *, const float *, const float *, float *,
                                             void *, hipStream_t);
template hipError_t launch_gram_apply<double>(const gct_plan *, const double *, const double *,
                                              double *, void *, hipStream_t);
template hipError_t launch_gram_spectrum<float>(const gct_plan *, const float *, float *, void *,
                                                hipStream_t);
template hipError_t launch_gram_spectrum<double>(const gct_plan *, const double *, double *, void *,
                                                 hipStream_t);
template hipError_t launch_apply_passes<float>(const gct_plan *, const float *, const float *,
                                               float *, void *, hipStream_t, const int64_t *,
                                               float *, const double *, const float *, double *);
template hipError_t launch_apply_passes<double>(const gct_plan *, const double *, const double *,
                                                double *, void *, hipStream_t, const int64_t *,
                                                double *, const double *, const double *, double *);

}  // namespace gct
