// Workgroup-level radix-2 FFTs in LDS, shared by the Gram-filter kernels.
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

__device__ __forceinline__ int brev(int v, int logP)
{
    return (int)(__brev((unsigned)v) >> (32 - logP));
}

// `nf` independent length-P transforms at buf + f*P.  Decimation in time:
// input in bit-reversed order, output in natural order.  tw[k] =
// e^{-2 pi i k / P}, k < P/2; INV selects the conjugate twiddles (unscaled
// inverse).  Every thread of the block must call it.
template <typename T, bool INV>
__device__ void fft_dit(C2<T> *buf, int logP, int nf, const C2<T> *__restrict__ tw)
{
    const int P = 1 << logP, hP = P >> 1;
    const int nb = nf * hP;
    for (int lh = 0; lh < logP; ++lh) {
        const int half = 1 << lh;
        const int tws = hP >> lh;
        for (int i = threadIdx.x; i < nb; i += blockDim.x) {
            const int f = i >> (logP - 1), b = i & (hP - 1);
            const int pos = b & (half - 1), grp = b >> lh;
            const int i0 = f * P + (grp << (lh + 1)) + pos, i1 = i0 + half;
            C2<T> w = tw[pos * tws];
            if (INV) w.y = -w.y;
            const C2<T> a = buf[i0];
            const C2<T> c = cmul(buf[i1], w);
            buf[i0] = {a.x + c.x, a.y + c.y};
            buf[i1] = {a.x - c.x, a.y - c.y};
        }
        __syncthreads();
    }
}

// Decimation in frequency: input in natural order, output bit-reversed.
template <typename T, bool INV>
__device__ void fft_dif(C2<T> *buf, int logP, int nf, const C2<T> *__restrict__ tw)
{
    const int P = 1 << logP, hP = P >> 1;
    const int nb = nf * hP;
    for (int lh = logP - 1; lh >= 0; --lh) {
        const int half = 1 << lh;
        const int tws = hP >> lh;
        for (int i = threadIdx.x; i < nb; i += blockDim.x) {
            const int f = i >> (logP - 1), b = i & (hP - 1);
            const int pos = b & (half - 1), grp = b >> lh;
            const int i0 = f * P + (grp << (lh + 1)) + pos, i1 = i0 + half;
            C2<T> w = tw[pos * tws];
            if (INV) w.y = -w.y;
            const C2<T> a = buf[i0], c = buf[i1];
            buf[i0] = {a.x + c.x, a.y + c.y};
            buf[i1] = cmul(C2<T>{a.x - c.x, a.y - c.y}, w);
        }
        __syncthreads();
    }
}

}  // namespace gct
