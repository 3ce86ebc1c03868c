// Group-level FFTs for the Gram-filtering kernels: register-blocked Stockham.
//
// Transform lengths P = 2^k or 3 * 2^k.  A length-P transform is owned by
// G = P/E threads; thread t holds E elements in registers in the strided
// layout v[q] = x[t + G q], q < E.  The transform runs as Stockham autosort
// passes: the first of radix E, then each of radix gcd(E, remaining length)
// (so every radix divides E), each thread computing E/R radix-R butterflies
// per pass in registers.  The first pass reads the registers directly (its
// butterfly inputs are exactly x[t + G r]); the last pass leaves its outputs
// in registers in the same strided layout; only the passes in between
// exchange through LDS.  So input and output need no permutation, a forward
// and an inverse transform can be chained in registers, and loads/stores of
// x[t + G q] are coalesced across a wave.
//
// E = 16 for P >= 1024 (one wave per 1024-point transform: passes 16, 16,
// 4), E = 8 for P = 512, E = 4 for P <= 256; for P = 3 * 2^k (1536 and 3072
// points) E = 24 (1536 points: passes 24, 8, 8) or 12, the radix-3 factor
// in the first pass.
#pragma once

#include <hip/hip_runtime.h>

namespace gct {

template <typename T>
struct C2 {
    T x, y;
};

// Transform length of a size code: 2^c for c < 32, 3 * 2^(c - 32) above.
__host__ __device__ constexpr int fft_size(int code) { return code < 32 ? 1 << code : 3 << (code - 32); }

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// cos and sin of 2 pi n / d at compile time (Taylor series after reduction
// to [-pi, pi]; the twiddles of the composite small DFTs)
constexpr double ctrig(double x, bool sine)
{
    const double pi = 3.14159265358979323846;
    while (x > pi) x -= 2 * pi;
    while (x < -pi) x += 2 * pi;
    double term = sine ? x : 1.0, sum = term;
    for (int i = sine ? 1 : 0; i < 40; i += 1) {
        const int a = sine ? 2 * i : 2 * i + 1, b = sine ? 2 * i + 1 : 2 * i + 2;
        term *= -x * x / ((double)a * (double)b);
        sum += term;
    }
    return sum;
}
constexpr double cos2pi(int n, int d) { return ctrig(2.0 * 3.14159265358979323846 * n / d, false); }
constexpr double sin2pi(int n, int d) { return ctrig(2.0 * 3.14159265358979323846 * n / d, true); }

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }

template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }

// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a)
{
    return INV ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
}

// e^{-+2 pi i m / P} from the half table tw[m] = e^{-2 pi i m / P}, m < P/2.
template <typename T, bool INV>
__device__ __forceinline__ C2<T> twid(const C2<T> *tw, int m, int hP)
{
    C2<T> w = m < hP ? tw[m] : C2<T>{-tw[m - hP].x, -tw[m - hP].y};
    if (INV) w.y = -w.y;
    return w;
}

// ---------------------------------------------------------------------------
// Small DFTs in registers, natural order in and out.
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ void dft2(C2<T> *v)
{
    const C2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4s(C2<T> &a0, C2<T> &a1, C2<T> &a2, C2<T> &a3)
{
    const C2<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
    const C2<T> t3 = mul_mi<T, INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(C2<T> *v)
{
    dft4s<T, INV>(v[0], v[1], v[2], v[3]);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(C2<T> *v)
{
    const T h = T(0.70710678118654752440);
    C2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4s<T, INV>(e0, e1, e2, e3);
    dft4s<T, INV>(o0, o1, o2, o3);
    // W8^1, W8^2, W8^3 (conjugated for the inverse)
    o1 = INV ? C2<T>{h * (o1.x - o1.y), h * (o1.x + o1.y)} : C2<T>{h * (o1.x + o1.y), h * (o1.y - o1.x)};
    o2 = mul_mi<T, INV>(o2);
    o3 = INV ? C2<T>{-h * (o3.x + o3.y), h * (o3.x - o3.y)} : C2<T>{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// v * e^{-+2 pi i J / 16} for a compile-time J in {1, 2, 3, 4, 6, 9}
template <typename T, bool INV, int J>
__device__ __forceinline__ C2<T> w16(C2<T> v)
{
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    constexpr double h = 0.70710678118654752440;
    constexpr double c = J == 1 ? c1 : J == 2 ? h : J == 3 ? s1 : J == 4 ? 0.0 : J == 6 ? -h : -c1;
    constexpr double s = J == 1 ? s1 : J == 2 ? h : J == 3 ? c1 : J == 4 ? 1.0 : J == 6 ? h : -s1;
    const C2<T> w = {T(c), INV ? T(s) : T(-s)};
    return cmul(v, w);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(C2<T> *v)
{
#pragma unroll
    for (int l = 0; l < 4; ++l) dft4s<T, INV>(v[l], v[4 + l], v[8 + l], v[12 + l]);
    // twiddle W16^{l m}: element 4 m + l holds Y_l[m]
    v[5] = w16<T, INV, 1>(v[5]);
    v[9] = w16<T, INV, 2>(v[9]);
    v[13] = w16<T, INV, 3>(v[13]);
    v[6] = w16<T, INV, 2>(v[6]);
    v[10] = w16<T, INV, 4>(v[10]);
    v[14] = w16<T, INV, 6>(v[14]);
    v[7] = w16<T, INV, 3>(v[7]);
    v[11] = w16<T, INV, 6>(v[11]);
    v[15] = w16<T, INV, 9>(v[15]);
    C2<T> o[16];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        C2<T> a0 = v[4 * m], a1 = v[4 * m + 1], a2 = v[4 * m + 2], a3 = v[4 * m + 3];
        dft4s<T, INV>(a0, a1, a2, a3);
        o[m] = a0;
        o[m + 4] = a1;
        o[m + 8] = a2;
        o[m + 12] = a3;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = o[q];
}

// 3-point DFT: with t = b + c, d = b - c and s = sin(2 pi / 3),
// X0 = a + t, X1,2 = a - t/2 -+ i s d (forward; signs swapped for the inverse)
template <typename T, bool INV>
__device__ __forceinline__ void dft3s(C2<T> &a, C2<T> &b, C2<T> &c)
{
    const T s = T(0.86602540378443864676);
    const C2<T> t = cadd(b, c), d = csub(b, c);
    const C2<T> m = {a.x - T(0.5) * t.x, a.y - T(0.5) * t.y};
    const C2<T> sd = mul_mi<T, INV>(C2<T>{s * d.x, s * d.y});  // -+ i s d
    a = cadd(a, t);
    b = cadd(m, sd);
    c = csub(m, sd);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(C2<T> *v);

// y[k1][n2] *= W_R^(n2 k1) for k1 = 1, 2 and n2 = 1 .. R2-1 (R = 3 R2), the
// factors evaluated at compile time
template <typename T, int R2, bool INV, int K1, int N2>
__device__ __forceinline__ void dft3x_twiddle(C2<T> (&y)[3][R2])
{
    if constexpr (K1 < 3) {
        if constexpr (N2 < R2) {
            constexpr double c = cos2pi(N2 * K1, 3 * R2), s = sin2pi(N2 * K1, 3 * R2);
            y[K1][N2] = cmul(y[K1][N2], C2<T>{T(c), INV ? T(s) : T(-s)});
            dft3x_twiddle<T, R2, INV, K1, N2 + 1>(y);
        } else {
            dft3x_twiddle<T, R2, INV, K1 + 1, 1>(y);
        }
    }
}

// Length 3 R2 (R2 = 1, 2, 4, 8), natural order in and out: n = R2 n1 + n2,
// k = k1 + 3 k2; 3-point DFTs over n1, twiddles W_R^(n2 k1), R2-point DFTs
// over n2.
template <typename T, int R2, bool INV>
__device__ __forceinline__ void dft3x(C2<T> *v)
{
    C2<T> y[3][R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        C2<T> a = v[n2], b = v[R2 + n2], c = v[2 * R2 + n2];
        dft3s<T, INV>(a, b, c);
        y[0][n2] = a;
        y[1][n2] = b;
        y[2][n2] = c;
    }
    dft3x_twiddle<T, R2, INV, 1, 1>(y);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        if constexpr (R2 > 1) dftR<T, R2, INV>(y[k1]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + 3 * k2] = y[k1][k2];
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(C2<T> *v)
{
    if constexpr (R == 1) return;
    else if constexpr (R % 3 == 0) dft3x<T, R / 3, INV>(v);
    else if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 4) dft4<T, INV>(v);
    else if constexpr (R == 8) dft8<T, INV>(v);
    else {
        static_assert(R == 16, "radix");
        dft16<T, INV>(v);
    }
}

// LDS layout of a transform: with ping-pong (two data areas of P entries
// where they fit in 64 KB with the twiddles) a pass reads one area and
// writes the other, so it needs one barrier instead of two.
template <typename T>
__host__ __device__ constexpr bool fft_pingpong(int P)
{
    return (size_t)(2 * P + P / 2) * sizeof(C2<T>) <= 32768;
}
template <typename T>
__host__ __device__ constexpr int fft_data_elems(int P)
{
    return fft_pingpong<T>(P) ? 2 * P : P;
}

// ---------------------------------------------------------------------------
// One Stockham pass of radix R on a length-P transform held by G = P/E
// threads.  FIRST: inputs are v (R == E, no twiddles); LAST: outputs go to v
// in the strided layout.  Otherwise x (LDS) is read and/or written: with PP
// the pass writes area A (x + A P) and reads the other one, else both in
// x.  Every thread of the block must call it (it contains barriers); after
// the LAST pass the whole LDS data area is free again.
// ---------------------------------------------------------------------------
template <typename T, int E, int P, int NS, int R, bool INV, bool FIRST, bool LAST, bool PP, int A>
__device__ __forceinline__ void fft_pass(C2<T> (&v)[E], C2<T> *x, int t, const C2<T> *tw)
{
    constexpr int B = E / R;
    constexpr int G = P / E;
    constexpr int stride = P / R;
    constexpr int tstep = P / (NS * R);
    constexpr int hP = P / 2;
    static_assert(E % R == 0 && P % (NS * R) == 0, "radix schedule");
    const C2<T> *xin = PP ? x + (A ^ 1) * P : x;
    C2<T> *xout = PP ? x + A * P : x;
    C2<T> u[E];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + G * b;
        const int k = j % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (FIRST) {
                u[b * R + r] = v[b * R + r];
            } else {
                C2<T> a = xin[j + r * stride];
                if (r > 0) a = cmul(a, twid<T, INV>(tw, r * k * tstep, hP));
                u[b * R + r] = a;
            }
        }
        dftR<T, R, INV>(&u[b * R]);
    }
    // every read of this pass is done before the area is written again (with
    // ping-pong the next write to it comes after the next pass's barrier)
    if constexpr (!FIRST && (!PP || LAST)) __syncthreads();
    if constexpr (LAST) {
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + B * r] = u[b * R + r];
    } else {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + G * b;
            const int k = j % NS;
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) xout[base + r * NS] = u[b * R + r];
        }
        __syncthreads();  // writes visible to the next pass
    }
}

template <typename T, int E, int P, int NS, bool INV, bool FIRST, bool PP = fft_pingpong<T>(P), int A = 0>
__device__ __forceinline__ void fft_passes(C2<T> (&v)[E], C2<T> *x, int t, const C2<T> *tw)
{
    constexpr int REM = P / NS;
    constexpr int R = cgcd(E, REM);  // E for the first pass (E divides P)
    constexpr bool LAST = REM == R;
    fft_pass<T, E, P, NS, R, INV, FIRST, LAST, PP, A>(v, x, t, tw);
    if constexpr (!LAST) fft_passes<T, E, P, NS * R, INV, false, PP, A ^ 1>(v, x, t, tw);
}

// Elements per thread for a length-P transform.
__host__ __device__ constexpr int fft_elems(int P)
{
    return P % 3 == 0 ? 24 : (P >= 1024 ? 16 : (P == 512 ? 8 : 4));
}

}  // namespace gct
