// Gram filtering (Sec. 4, closing remark): H^T H is Toeplitz-block-Toeplitz,
// so y = H^T H c is the zero-padded linear convolution of the N x N
// coefficients with the (2N-1)^2 Gram filter.  It is evaluated exactly (up
// to rounding) through the P x P circulant embedding, P >= 2N-1 a power of
// two: y = IFFT2(Ghat . FFT2(c_padded))[0:N, 0:N], with Ghat real and even
// because G[k] = G[-k].
//
// Three passes, each a block-local FFT (fft_common.h):
//   rows:    pairs of image rows -> one complex FFT -> two real-row spectra,
//            written transposed as W1[w1][k2], w1 in [0, P/2];
//   columns: per w1, FFT along k2 (N nonzero of P), times Ghat[w1][.],
//            inverse FFT, keep k2 < N -> W2[w1][k2];
//   rows:    pairs of Hermitian row spectra -> one complex inverse FFT ->
//            two real output rows, keep k1 < N.
// The 1/P^2 normalisation is folded into Ghat.  One block of P/E threads
// owns one transform (a single wave for P = 1024).
#include <algorithm>

#include "fft_common.h"
#include "gct_internal.h"

namespace gct {

// Status word of a running CG solve (see cg.hip): kernels return at once
// when it is non-zero, so iterations queued after convergence cost only a
// launch.
__device__ __forceinline__ bool halted(const int64_t *status) { return status && *status != 0; }

// Twiddles go to LDS after the data area when both fit in 64 KB, else they
// are read from the plan's global table.
template <typename T>
__host__ __device__ constexpr bool twiddles_in_lds(int P)
{
    return (size_t)(P + P / 2) * sizeof(C2<T>) <= 65536;
}

template <typename T, bool TWL>
__device__ __forceinline__ const C2<T> *stage_twiddles(C2<T> *lds_after_data,
                                                       const C2<T> *__restrict__ tw, int hP)
{
    if (!TWL) return tw;
    for (int i = threadIdx.x; i < hP; i += blockDim.x) lds_after_data[i] = tw[i];
    return lds_after_data;
}

// One transform per block: G = P/E threads, thread t holds x[t + G q].
// ---------------------------------------------------------------------------
// Pass 1: forward real FFT of a pair of image rows.  With `pupd` set (CG),
// the rows are first updated in place as p = r + beta p (beta from *beta).
// ---------------------------------------------------------------------------
template <typename T, int LOGP>
__global__ void __launch_bounds__(256)
k_rows_fwd(const T *__restrict__ src, C2<T> *__restrict__ W1, int N,
           const C2<T> *__restrict__ tw, const int64_t *status, T *pupd, const double *beta)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int P = 1 << LOGP, hP = P >> 1, E = fft_elems(P), G = P / E;
    constexpr bool TWL = twiddles_in_lds<T>(P);
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int t = threadIdx.x;
    const int ra = 2 * blockIdx.x, rb = ra + 1;
    const T bt = pupd ? (T)(*beta) : T(0);
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = t + G * q;
        T re = 0, im = 0;
        if (n < N) {
            const size_t ia = (size_t)ra * N + n, ib = (size_t)rb * N + n;
            re = src[ia];
            if (rb < N) im = src[ib];
            if (pupd) {
                re += bt * pupd[ia];
                pupd[ia] = re;
                if (rb < N) {
                    im += bt * pupd[ib];
                    pupd[ib] = im;
                }
            }
        }
        v[q] = {re, im};
    }
    const C2<T> *tws = stage_twiddles<T, TWL>(x + P, tw, hP);
    if (TWL) __syncthreads();
    fft_strided<T, LOGP, false>(v, x, t, tws);
    // split the two real rows: Xa = (Z[k] + conj Z[-k])/2, Xb = (Z[k] - conj Z[-k])/(2i)
#pragma unroll
    for (int q = 0; q < E; ++q) x[t + G * q] = v[q];
    __syncthreads();
    for (int k = t; k <= hP; k += G) {
        const C2<T> Zk = x[k], Zm = x[(P - k) & (P - 1)];
        W1[(size_t)k * N + ra] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        if (rb < N) W1[(size_t)k * N + rb] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
    }
}

// ---------------------------------------------------------------------------
// Pass 2: per frequency column w1: FFT along k2, multiply by the real
// spectrum, inverse FFT (all in registers between the two), keep the first
// N entries.
// ---------------------------------------------------------------------------
template <typename T, int LOGP>
__global__ void __launch_bounds__(256)
k_cols(const C2<T> *__restrict__ W1, C2<T> *__restrict__ W2, const T *__restrict__ Ghat, int N,
       const C2<T> *__restrict__ tw, const int64_t *status)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int P = 1 << LOGP, hP = P >> 1, E = fft_elems(P), G = P / E;
    constexpr bool TWL = twiddles_in_lds<T>(P);
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int t = threadIdx.x;
    const int col = blockIdx.x;  // in [0, P/2]
    const C2<T> *in = W1 + (size_t)col * N;
    const T *g = Ghat + (size_t)col * P;
    C2<T> v[E];
    T gs[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = t + G * q;
        v[q] = n < N ? in[n] : C2<T>{T(0), T(0)};
        gs[q] = g[n];
    }
    const C2<T> *tws = stage_twiddles<T, TWL>(x + P, tw, hP);
    if (TWL) __syncthreads();
    fft_strided<T, LOGP, false>(v, x, t, tws);
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = {v[q].x * gs[q], v[q].y * gs[q]};
    fft_strided<T, LOGP, true>(v, x, t, tws);
    C2<T> *out = W2 + (size_t)col * N;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = t + G * q;
        if (n < N) out[n] = v[q];
    }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse real FFT of a pair of row spectra.  With `dotv` set (CG),
// each block also writes the FP64 partial sum of dotv . y over its rows.
// ---------------------------------------------------------------------------
template <typename T, int LOGP>
__global__ void __launch_bounds__(256)
k_rows_inv(const C2<T> *__restrict__ W2, T *__restrict__ y, int N,
           const C2<T> *__restrict__ tw, const int64_t *status, const T *__restrict__ dotv,
           double *__restrict__ partial)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int P = 1 << LOGP, hP = P >> 1, E = fft_elems(P), G = P / E;
    constexpr bool TWL = twiddles_in_lds<T>(P);
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int t = threadIdx.x;
    const int ra = 2 * blockIdx.x, rb = ra + 1;
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int k = t + G * q;
        const int kk = k <= hP ? k : P - k;  // Hermitian extension
        C2<T> Ya = W2[(size_t)kk * N + ra];
        C2<T> Yb = rb < N ? W2[(size_t)kk * N + rb] : C2<T>{T(0), T(0)};
        if (k > hP) {
            Ya.y = -Ya.y;
            Yb.y = -Yb.y;
        }
        v[q] = {Ya.x - Yb.y, Ya.y + Yb.x};
    }
    const C2<T> *tws = stage_twiddles<T, TWL>(x + P, tw, hP);
    if (TWL) __syncthreads();
    fft_strided<T, LOGP, true>(v, x, t, tws);
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = t + G * q;
        if (n >= N) continue;
        y[(size_t)ra * N + n] = v[q].x;
        if (dotv) acc += (double)dotv[(size_t)ra * N + n] * (double)v[q].x;
        if (rb < N) {
            y[(size_t)rb * N + n] = v[q].y;
            if (dotv) acc += (double)dotv[(size_t)rb * N + n] * (double)v[q].y;
        }
    }
    if (partial) {
        // reuse the LDS area (the launcher sizes it to >= blockDim doubles)
        __syncthreads();
        double *red = reinterpret_cast<double *>(smem_raw);
        red[t] = acc;
        __syncthreads();
        for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
            if (t < s) red[t] += red[t + s];
            __syncthreads();
        }
        if (t == 0) partial[blockIdx.x] = red[0];
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

template <typename T, int LOGP>
__global__ void __launch_bounds__(256)
k_spec_rows(const T *__restrict__ G, C2<T> *__restrict__ R, int N,
            const C2<T> *__restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int P = 1 << LOGP, hP = P >> 1, E = fft_elems(P), Gt = P / E;
    constexpr bool TWL = twiddles_in_lds<T>(P);
    const int W = 2 * N - 1;
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int t = threadIdx.x;
    const int seq = blockIdx.x;  // embedded row pair (2 seq, 2 seq + 1), < P/2
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
    const C2<T> *tws = stage_twiddles<T, TWL>(x + P, tw, hP);
    if (TWL) __syncthreads();
    fft_strided<T, LOGP, false>(v, x, t, tws);
#pragma unroll
    for (int q = 0; q < E; ++q) x[t + Gt * q] = v[q];
    __syncthreads();
    for (int k = t; k <= hP; k += Gt) {
        const C2<T> Zk = x[k], Zm = x[(P - k) & (P - 1)];
        R[(size_t)k * P + 2 * seq] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        R[(size_t)k * P + 2 * seq + 1] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
    }
}

template <typename T, int LOGP>
__global__ void __launch_bounds__(256)
k_spec_cols(const C2<T> *__restrict__ R, T *__restrict__ Ghat,
            const C2<T> *__restrict__ tw, T scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int P = 1 << LOGP, hP = P >> 1, E = fft_elems(P), Gt = P / E;
    constexpr bool TWL = twiddles_in_lds<T>(P);
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int t = threadIdx.x;
    const int col = blockIdx.x;
    C2<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = R[(size_t)col * P + t + Gt * q];
    const C2<T> *tws = stage_twiddles<T, TWL>(x + P, tw, hP);
    if (TWL) __syncthreads();
    fft_strided<T, LOGP, false>(v, x, t, tws);
#pragma unroll
    for (int q = 0; q < E; ++q) Ghat[(size_t)col * P + t + Gt * q] = v[q].x * scale;
}

// ---------------------------------------------------------------------------
// Launch geometry: one transform per block, P/E threads.
// ---------------------------------------------------------------------------
struct FftCfg {
    int threads;   // P / E
    size_t lds;    // bytes of dynamic LDS
};

template <typename T>
static FftCfg fft_cfg(int logP)
{
    FftCfg c;
    const int P = 1 << logP;
    c.threads = P / fft_elems(P);
    c.lds = (size_t)P * sizeof(C2<T>) + (twiddles_in_lds<T>(P) ? (size_t)(P / 2) * sizeof(C2<T>) : 0);
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

int apply_row_blocks(const gct_plan *p, size_t /*elem*/) { return (p->N + 1) / 2; }

// Dispatch on log2 P (4 .. 4096).
#define GCT_LAUNCH_FFT(kern, T, logP, cfg, grid, s, ...)                                        \
    do {                                                                                       \
        const dim3 blk_(cfg.threads);                                                          \
        switch (logP) {                                                                        \
        case 2: hipLaunchKernelGGL((kern<T, 2>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 3: hipLaunchKernelGGL((kern<T, 3>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 4: hipLaunchKernelGGL((kern<T, 4>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 5: hipLaunchKernelGGL((kern<T, 5>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 6: hipLaunchKernelGGL((kern<T, 6>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 7: hipLaunchKernelGGL((kern<T, 7>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 8: hipLaunchKernelGGL((kern<T, 8>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 9: hipLaunchKernelGGL((kern<T, 9>), grid, blk_, cfg.lds, s, __VA_ARGS__); break;  \
        case 10: hipLaunchKernelGGL((kern<T, 10>), grid, blk_, cfg.lds, s, __VA_ARGS__); break; \
        case 11: hipLaunchKernelGGL((kern<T, 11>), grid, blk_, cfg.lds, s, __VA_ARGS__); break; \
        default: hipLaunchKernelGGL((kern<T, 12>), grid, blk_, cfg.lds, s, __VA_ARGS__); break; \
        }                                                                                      \
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
    const dim3 rgrid((N + 1) / 2), cgrid(P / 2 + 1);
    GCT_LAUNCH_FFT(k_rows_fwd, T, logP, c, rgrid, s, src, W1, N, tw, status, pupd, beta);
    GCT_LAUNCH_FFT(k_cols, T, logP, c, cgrid, s, W1, W2, Ghat, N, tw, status);
    GCT_LAUNCH_FFT(k_rows_inv, T, logP, c, rgrid, s, W2, y, N, tw, status, dotv, partial);
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
    GCT_LAUNCH_FFT(k_spec_rows, T, logP, c, dim3(P / 2), s, G, R, N, tw);
    const T scale = T(1.0 / ((double)P * (double)P));
    GCT_LAUNCH_FFT(k_spec_cols, T, logP, c, dim3(P / 2 + 1), s, R, Ghat, tw, scale);
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
