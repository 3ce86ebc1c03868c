// Gram filtering (Sec. 4, closing remark): H^T H is Toeplitz-block-Toeplitz,
// so y = H^T H c is the zero-padded linear convolution of the N x N
// coefficients with the (2N-1)^2 Gram filter.  It is evaluated exactly (up
// to rounding) through the P x P circulant embedding, P >= 2N-1 a power of
// two: y = IFFT2(Ghat . FFT2(c_padded))[0:N, 0:N], with Ghat real and even
// because G[k] = G[-k].
//
// Three passes, each a workgroup-local FFT in LDS:
//   rows:    pairs of image rows -> one complex FFT -> two real-row spectra,
//            written transposed as W1[w1][k2], w1 in [0, P/2];
//   columns: per w1, FFT along k2 (N nonzero of P), times Ghat[w1][.],
//            inverse FFT, keep k2 < N -> W2[w1][k2];
//   rows:    pairs of Hermitian row spectra -> one complex inverse FFT ->
//            two real output rows, keep k1 < N.
// The 1/P^2 normalisation is folded into Ghat.
#include <algorithm>

#include "fft_common.h"
#include "gct_internal.h"

namespace gct {

// Status word of a running CG solve (see cg.hip): kernels return at once
// when it is non-zero, so iterations queued after convergence cost only a
// launch.
__device__ __forceinline__ bool halted(const int64_t *status) { return status && *status != 0; }

// ---------------------------------------------------------------------------
// Pass 1: forward real FFT of image rows.  With `pupd` set (CG), the row
// vector is first updated in place as p = r + beta p (beta read from *beta).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_rows_fwd(const T *__restrict__ src, C2<T> *__restrict__ W1, int N, int logP, int nf,
           const C2<T> *__restrict__ tw, const int64_t *status, T *pupd, const double *beta)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const int P = 1 << logP;
    const int row0 = blockIdx.x * 2 * nf;
    const T bt = pupd ? (T)(*beta) : T(0);
    for (int i = threadIdx.x; i < nf * P; i += blockDim.x) {
        const int f = i >> logP, n = i & (P - 1);
        const int ra = row0 + 2 * f, rb = ra + 1;
        T re = 0, im = 0;
        if (n < N) {
            if (ra < N) {
                if (pupd) {
                    re = src[(size_t)ra * N + n] + bt * pupd[(size_t)ra * N + n];
                    pupd[(size_t)ra * N + n] = re;
                } else {
                    re = src[(size_t)ra * N + n];
                }
            }
            if (rb < N) {
                if (pupd) {
                    im = src[(size_t)rb * N + n] + bt * pupd[(size_t)rb * N + n];
                    pupd[(size_t)rb * N + n] = im;
                } else {
                    im = src[(size_t)rb * N + n];
                }
            }
        }
        buf[f * P + brev(n, logP)] = {re, im};
    }
    __syncthreads();
    fft_dit<T, false>(buf, logP, nf, tw);
    const int hP1 = (P >> 1) + 1;
    for (int i = threadIdx.x; i < nf * hP1; i += blockDim.x) {
        const int f = i / hP1, k = i - f * hP1;
        const C2<T> Zk = buf[f * P + k], Zm = buf[f * P + ((P - k) & (P - 1))];
        const int ra = row0 + 2 * f;
        if (ra < N) W1[(size_t)k * N + ra] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        if (ra + 1 < N) W1[(size_t)k * N + ra + 1] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
    }
}

// ---------------------------------------------------------------------------
// Pass 2: per frequency column w1: FFT along k2, multiply by the real
// spectrum, inverse FFT, keep the first N entries.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_cols(const C2<T> *__restrict__ W1, C2<T> *__restrict__ W2, const T *__restrict__ Ghat, int N,
       int logP, const C2<T> *__restrict__ tw, const int64_t *status)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const int P = 1 << logP;
    const int k = blockIdx.x;  // in [0, P/2]
    const C2<T> *col = W1 + (size_t)k * N;
    for (int n = threadIdx.x; n < P; n += blockDim.x)
        buf[brev(n, logP)] = n < N ? col[n] : C2<T>{T(0), T(0)};
    __syncthreads();
    fft_dit<T, false>(buf, logP, 1, tw);
    const T *g = Ghat + (size_t)k * P;
    for (int n = threadIdx.x; n < P; n += blockDim.x) {
        const T s = g[n];
        buf[n] = {buf[n].x * s, buf[n].y * s};
    }
    __syncthreads();
    fft_dif<T, true>(buf, logP, 1, tw);
    C2<T> *out = W2 + (size_t)k * N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) out[n] = buf[brev(n, logP)];
}

// ---------------------------------------------------------------------------
// Pass 3: inverse real FFT of row spectra.  With `dotv` set (CG), each block
// also writes the FP64 partial sum of dotv . y over its rows.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_rows_inv(const C2<T> *__restrict__ W2, T *__restrict__ y, int N, int logP, int nf,
           const C2<T> *__restrict__ tw, const int64_t *status, const T *__restrict__ dotv,
           double *__restrict__ partial)
{
    if (halted(status)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const int P = 1 << logP, hP = P >> 1;
    const int row0 = blockIdx.x * 2 * nf;
    for (int i = threadIdx.x; i < nf * P; i += blockDim.x) {
        const int f = i >> logP, k = i & (P - 1);
        const int ra = row0 + 2 * f, rb = ra + 1;
        C2<T> Ya = {T(0), T(0)}, Yb = {T(0), T(0)};
        if (k <= hP) {
            if (ra < N) Ya = W2[(size_t)k * N + ra];
            if (rb < N) Yb = W2[(size_t)k * N + rb];
        } else {
            if (ra < N) { Ya = W2[(size_t)(P - k) * N + ra]; Ya.y = -Ya.y; }
            if (rb < N) { Yb = W2[(size_t)(P - k) * N + rb]; Yb.y = -Yb.y; }
        }
        buf[i] = {Ya.x - Yb.y, Ya.y + Yb.x};
    }
    __syncthreads();
    fft_dif<T, true>(buf, logP, nf, tw);
    double acc = 0.0;
    for (int i = threadIdx.x; i < nf * N; i += blockDim.x) {
        const int f = i / N, n = i - f * N;
        const int ra = row0 + 2 * f, rb = ra + 1;
        const C2<T> v = buf[f * P + brev(n, logP)];
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
        // reuse the transform buffer (the launcher sizes it to >= 256 doubles)
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
__device__ __forceinline__ int embed_tap(int q, int N, int P)
{
    if (q <= N - 1) return q;
    if (q >= P - N + 1) return q - P;
    return 1 << 30;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_spec_rows(const T *__restrict__ G, C2<T> *__restrict__ R, int N, int logP, int nf,
            const C2<T> *__restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const int P = 1 << logP, W = 2 * N - 1;
    const int row0 = blockIdx.x * 2 * nf;  // embedded rows q2 in [0, P)
    for (int i = threadIdx.x; i < nf * P; i += blockDim.x) {
        const int f = i >> logP, q1 = i & (P - 1);
        const int k1 = embed_tap(q1, N, P);
        T re = 0, im = 0;
        if (k1 != (1 << 30)) {
            const int ka = embed_tap(row0 + 2 * f, N, P), kb = embed_tap(row0 + 2 * f + 1, N, P);
            if (ka != (1 << 30)) re = G[(size_t)(ka + N - 1) * W + (k1 + N - 1)];
            if (kb != (1 << 30)) im = G[(size_t)(kb + N - 1) * W + (k1 + N - 1)];
        }
        buf[f * P + brev(q1, logP)] = {re, im};
    }
    __syncthreads();
    fft_dit<T, false>(buf, logP, nf, tw);
    const int hP1 = (P >> 1) + 1;
    for (int i = threadIdx.x; i < nf * hP1; i += blockDim.x) {
        const int f = i / hP1, k = i - f * hP1;
        const C2<T> Zk = buf[f * P + k], Zm = buf[f * P + ((P - k) & (P - 1))];
        const int ra = row0 + 2 * f;
        R[(size_t)k * P + ra] = {(Zk.x + Zm.x) * T(0.5), (Zk.y - Zm.y) * T(0.5)};
        R[(size_t)k * P + ra + 1] = {(Zk.y + Zm.y) * T(0.5), (Zm.x - Zk.x) * T(0.5)};
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_spec_cols(const C2<T> *__restrict__ R, T *__restrict__ Ghat, int logP,
            const C2<T> *__restrict__ tw, T scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
    const int P = 1 << logP;
    const int k = blockIdx.x;
    for (int n = threadIdx.x; n < P; n += blockDim.x) buf[brev(n, logP)] = R[(size_t)k * P + n];
    __syncthreads();
    fft_dit<T, false>(buf, logP, 1, tw);
    for (int n = threadIdx.x; n < P; n += blockDim.x) Ghat[(size_t)k * P + n] = buf[n].x * scale;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
static int rows_per_fft_block(int P)
{
    // transforms per block: about 32 KB of LDS, at most 8, at most P/2 so
    // that 2 nf rows divide the P embedded rows of the spectrum pass
    int nf = 32768 / (P * (int)sizeof(C2<T>));
    if (nf > 8) nf = 8;
    if (nf > P / 2) nf = P / 2;
    return nf < 1 ? 1 : nf;
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

// The three passes of one apply; status/pupd/beta/dotv/partial are the CG
// hooks (all null for a plain apply).
template <typename T>
hipError_t launch_apply_passes(const gct_plan *p, const T *Ghat, const T *src, T *y, void *ws,
                               hipStream_t s, const int64_t *status, T *pupd, const double *beta,
                               const T *dotv, double *partial)
{
    const int N = p->N, P = p->P, logP = p->logP;
    const int nf = rows_per_fft_block<T>(P);
    const size_t w1 = align256((size_t)(P / 2 + 1) * N * 2 * sizeof(T));
    C2<T> *W1 = reinterpret_cast<C2<T> *>(ws);
    C2<T> *W2 = reinterpret_cast<C2<T> *>(reinterpret_cast<char *>(ws) + w1);
    const C2<T> *tw = twiddles<T>(p);
    const int rblocks = (N + 2 * nf - 1) / (2 * nf);
    const size_t lds_rows = (size_t)nf * P * sizeof(C2<T>), lds_col = (size_t)P * sizeof(C2<T>);
    hipLaunchKernelGGL(k_rows_fwd<T>, dim3(rblocks), dim3(256), lds_rows, s, src, W1, N, logP, nf,
                       tw, status, pupd, beta);
    hipLaunchKernelGGL(k_cols<T>, dim3(P / 2 + 1), dim3(256), lds_col, s, W1, W2, Ghat, N, logP, tw,
                       status);
    hipLaunchKernelGGL(k_rows_inv<T>, dim3(rblocks), dim3(256), std::max(lds_rows, (size_t)256 * sizeof(double)), s, W2, y, N, logP, nf, tw,
                       status, dotv, partial);
    return hipGetLastError();
}

int apply_row_blocks(const gct_plan *p, size_t elem)
{
    const int nf = elem == 4 ? rows_per_fft_block<float>(p->P) : rows_per_fft_block<double>(p->P);
    return (p->N + 2 * nf - 1) / (2 * nf);
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
    const int nf = rows_per_fft_block<T>(P);
    C2<T> *R = reinterpret_cast<C2<T> *>(ws);
    const C2<T> *tw = twiddles<T>(p);
    const int rblocks = P / (2 * nf);  // P is a power of two >= 4 and 2 nf divides it
    hipLaunchKernelGGL(k_spec_rows<T>, dim3(rblocks), dim3(256), (size_t)nf * P * sizeof(C2<T>), s,
                       G, R, N, logP, nf, tw);
    const T scale = T(1.0 / ((double)P * (double)P));
    hipLaunchKernelGGL(k_spec_cols<T>, dim3(P / 2 + 1), dim3(256), (size_t)P * sizeof(C2<T>), s, R,
                       Ghat, logP, tw, scale);
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
