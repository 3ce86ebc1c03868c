// Workgroup-level FFTs in LDS, shared by the Gram-filter kernels.
//
// Mixed radix-4/2 Stockham autosort transform, natural order in and out,
// computed in place: each thread owns one radix-4 butterfly per stage (two
// radix-2 butterflies in the final stage when log2 P is odd), reads its four
// inputs, waits for the whole group, then writes its four outputs.  A
// length-P transform therefore uses P/4 threads and log4(P) (+1) stages.
#pragma once

#include <hip/hip_runtime.h>

namespace gct {

template <typename T>
struct C2 {
    T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }

template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }

// e^{-+2 pi i m / P} from the half table tw[m] = e^{-2 pi i m / P}, m < P/2.
template <typename T, bool INV>
__device__ __forceinline__ C2<T> twid(const C2<T> *tw, int m, int hP)
{
    C2<T> w = m < hP ? tw[m] : C2<T>{-tw[m - hP].x, -tw[m - hP].y};
    if (INV) w.y = -w.y;
    return w;
}

// One length-P transform on x[0..P) by the P/4 threads t = 0..P/4-1 of a
// group; every thread of the block must call it (it contains barriers).
// Forward uses e^{-2 pi i nk/P}; INV the conjugate, unscaled.
template <typename T, bool INV>
__device__ void fft_inplace(C2<T> *x, int logP, int t, const C2<T> *tw)
{
    const int P = 1 << logP, Q = P >> 2, hP = P >> 1;
    int Ns = 1, lNs = 0, rem = logP;
    while (rem >= 2) {
        const int k = t & (Ns - 1);
        const int stride = P >> (lNs + 2);
        C2<T> v0 = x[t], v1 = x[t + Q], v2 = x[t + 2 * Q], v3 = x[t + 3 * Q];
        v1 = cmul(v1, twid<T, INV>(tw, k * stride, hP));
        v2 = cmul(v2, twid<T, INV>(tw, 2 * k * stride, hP));
        v3 = cmul(v3, twid<T, INV>(tw, 3 * k * stride, hP));
        const C2<T> t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = csub(v1, v3);
        // multiply t3 by -i (forward) or +i (inverse)
        const C2<T> t3r = INV ? C2<T>{-t3.y, t3.x} : C2<T>{t3.y, -t3.x};
        __syncthreads();
        const int base = ((t - k) << 2) + k;
        x[base] = cadd(t0, t2);
        x[base + Ns] = cadd(t1, t3r);
        x[base + 2 * Ns] = csub(t0, t2);
        x[base + 3 * Ns] = csub(t1, t3r);
        __syncthreads();
        Ns <<= 2;
        lNs += 2;
        rem -= 2;
    }
    if (rem == 1) {
        const int stride = P >> (lNs + 1);
        C2<T> A[2], B[2];
        int kk[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = t + q * Q;
            const int k = j & (Ns - 1);
            kk[q] = k;
            const C2<T> a = x[j];
            const C2<T> b = cmul(x[j + hP], twid<T, INV>(tw, k * stride, hP));
            A[q] = cadd(a, b);
            B[q] = csub(a, b);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = t + q * Q;
            const int base = ((j - kk[q]) << 1) + kk[q];
            x[base] = A[q];
            x[base + Ns] = B[q];
        }
        __syncthreads();
    }
}

}  // namespace gct
