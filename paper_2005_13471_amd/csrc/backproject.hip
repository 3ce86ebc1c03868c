// Sinogram interpolation, exact-adjoint back projection and the forward
// model (Sec. 2, Sec. 4, Sec. 5).
#include <algorithm>
#include <cmath>

#include "gct_internal.h"

namespace gct {

// ---------------------------------------------------------------------------
// Correction filter (Sec. 5, eq. correction filter).  One thread per output
// element p[a][m + K], m in [-K, M-1+K]; rows whose B-spline degree is 0 or 1
// are copied (q = delta), degree-2 rows are filtered with the 2K+1 taps.
// A block first stages the 256 + 2K input samples its outputs reach into LDS
// (zero outside the row), so the taps read LDS instead of 2K+1 global loads
// per output; the terms are summed in ascending tap order, and the zero
// samples add exact zeros, so the result equals the plain truncated sum.
// KC: the truncation K fixed at compile time (the default 40: the tap loop
// unrolls and the taps are loaded once per wave, not once per term), or 0
// (K at run time).
// ---------------------------------------------------------------------------
template <typename T, int KC>
__global__ void __launch_bounds__(256)
k_prefilter(const T *__restrict__ g, T *__restrict__ out, int n, int M, int Kr,
            const T *__restrict__ q, const int32_t *__restrict__ deg)
{
    const int K = KC > 0 ? KC : Kr;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *s_row = reinterpret_cast<T *>(smem_raw);  // row[m0 - 2K .. m0 + 255]
    const int Mp = M + 2 * K;
    const int a = blockIdx.y;
    const int mo0 = blockIdx.x * blockDim.x;
    const int mo = mo0 + threadIdx.x;
    const T *row = g + (size_t)a * M;
    if (deg[a] != 2) {  // uniform per block
        if (mo < Mp) {
            const int m = mo - K;
            out[(size_t)a * Mp + mo] = (m >= 0 && m < M) ? row[m] : T(0);
        }
        return;
    }
    // s_row[i] = row[mo0 - 2K + i] (output mo uses m - j = mo - K - j, j in [-K, K])
    const int span = blockDim.x + 2 * K;
    for (int i = threadIdx.x; i < span; i += blockDim.x) {
        const int src = mo0 - 2 * K + i;
        s_row[i] = (src >= 0 && src < M) ? row[src] : T(0);
    }
    __syncthreads();
    if (mo >= Mp) return;
    // term j reads row[mo - K - j] = s_row[threadIdx.x + K - j]
    const T *w = s_row + threadIdx.x + K;
    T acc = 0;
    if constexpr (KC > 0) {
#pragma unroll
        for (int j = -KC; j <= KC; ++j) acc += q[j + KC] * w[-j];
    } else {
        for (int j = -K; j <= K; ++j) acc += q[j + K] * w[-j];
    }
    out[(size_t)a * Mp + mo] = acc;
}

template <typename T>
hipError_t launch_prefilter(const gct_plan *p, const T *g, T *out, hipStream_t s)
{
    const int Mp = p->M + 2 * p->K;
    const dim3 grid((Mp + 255) / 256, p->n);
    const size_t lds = (size_t)(256 + 2 * p->K) * sizeof(T);
    if (lds > 64 * 1024) return hipErrorInvalidConfiguration;
    const T *q = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.q_f32 : p->dev.q_f64);
    const int32_t *deg = reinterpret_cast<const int32_t *>(p->dev.deg);
    if (p->K == 40)
        hipLaunchKernelGGL((k_prefilter<T, 40>), grid, dim3(256), lds, s, g, out, p->n, p->M, p->K, q, deg);
    else
        hipLaunchKernelGGL((k_prefilter<T, 0>), grid, dim3(256), lds, s, g, out, p->n, p->M, p->K, q, deg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Back projection (Sec. 5).  b[k] = sum_theta sum_m p[m] kappa_theta(m - z_k)
// with z_k the pixel centre's projection in fractional bin units and
// kappa_theta = l1 l2 M_{Xi/lambda_y}, Xi = {l1|c|, l2|s|, zeta,
// lambda_y x (d+1)}: the exact integral of the pixel footprint against the
// B-spline basis of the interpolated sinogram.
//
// On each sub-interval s of t = z - floor(z), kappa(j - t) is a polynomial
// in t with coefficients C[s][j][.] (built on the host in FP64: exact in the
// offset from the sub-interval's start brk[s], then re-expanded in powers of
// t, so that no breakpoint is subtracted per pixel), so the whole angle's
// contribution is the piecewise polynomial
//   S(z) = sum_k t^k E[m0][s][k],  E[m][s][k] = sum_j p[m + jlo + j] C[s][j][k],
// m0 = floor(z).  A block owns a TILE x TILE pixel tile; per angle it forms E
// for the few bins the tile projects onto (in LDS), then every pixel finds
// its (m0, s) and evaluates one polynomial.  FP64 is used only for z.
// ---------------------------------------------------------------------------
// Per-angle variant (kept for kernels whose tables exceed the chunked
// kernel's LDS budget): tables of CH angles are staged together, E is
// double-buffered so each angle costs one barrier.
struct BPLayout {
    int tile, rmax, ch;
    size_t lds;
};

template <typename T, int TILE>
__global__ void __launch_bounds__(TILE * TILE)
k_backproject(const T *__restrict__ pf, T *__restrict__ b, int N, int n, int Mp, int K,
              const double *__restrict__ geo, const int32_t *__restrict__ ints,
              const T *__restrict__ brk, const T *__restrict__ coef, int smax, int J, int D1,
              int rmax, int CH)
{
    constexpr int NT = TILE * TILE;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per_coef = smax * J * D1;
    const int pseg = rmax + J;
    const int eblk = rmax * smax * D1;
    T *s_E = reinterpret_cast<T *>(smem_raw);  // [2][rmax][smax][D1]
    T *s_C = s_E + 2 * eblk;                   // [CH][smax][J][D1]
    T *s_p = s_C + CH * per_coef;              // [CH][rmax + J]
    T *s_b = s_p + CH * pseg;                  // [CH][smax]
    const int tid = threadIdx.x;
    const int k1a = blockIdx.x * TILE, k2a = blockIdx.y * TILE;
    const int k1 = k1a + tid % TILE, k2 = k2a + tid / TILE;
    const double kx0 = k1a, kx1 = k1a + TILE - 1, ky0 = k2a, ky1 = k2a + TILE - 1;
    // bin window of the tile at angle a: [mlo, mlo + R) (one bin of margin
    // each side against rounding of z)
    auto window = [&](int a, int &mlo, int &R) {
        const double z0 = geo[4 * a], dz1 = geo[4 * a + 1], dz2 = geo[4 * a + 2];
        const double e1 = kx0 * dz1, e2 = kx1 * dz1, f1 = ky0 * dz2, f2 = ky1 * dz2;
        const double zmin = z0 + fmin(e1, e2) + fmin(f1, f2);
        const double zmax = z0 + fmax(e1, e2) + fmax(f1, f2);
        mlo = (int)floor(zmin) - 1;
        R = min((int)floor(zmax) + 2 - mlo, rmax);
    };
    T acc = 0, comp = 0;
    int parity = 0;
    for (int a0 = 0; a0 < n; a0 += CH) {
        const int cnt = min(CH, n - a0);
        __syncthreads();  // previous chunk done with s_C / s_p / s_b
        for (int i = tid; i < cnt * per_coef; i += NT) s_C[i] = coef[(size_t)a0 * per_coef + i];
        for (int i = tid; i < cnt * smax; i += NT) s_b[i] = brk[(size_t)a0 * smax + i];
        for (int i = tid; i < cnt * pseg; i += NT) {
            const int c = i / pseg, off = i - c * pseg;
            const int a = a0 + c;
            int mlo, R;
            window(a, mlo, R);
            const int mi = mlo + ints[4 * a + 1] + off + K;
            s_p[i] = (off < R + J - 1 && mi >= 0 && mi < Mp) ? pf[(size_t)a * Mp + mi] : T(0);
        }
        __syncthreads();
        for (int c = 0; c < cnt; ++c) {
            const int a = a0 + c;
            const int nsub = ints[4 * a];
            int mlo, R;
            window(a, mlo, R);
            T *E = s_E + parity * eblk;
            const T *Cc = s_C + c * per_coef;
            const T *pc = s_p + c * pseg;
            const int nE = R * nsub * D1;
            for (int i = tid; i < nE; i += NT) {
                const int k = i % D1, rest = i / D1;
                const int sidx = rest % nsub, mi = rest / nsub;
                const T *cf = Cc + sidx * J * D1 + k;
                const T *pp = pc + mi;
                T e = 0;
                for (int j = 0; j < J; ++j) e += pp[j] * cf[j * D1];
                E[i] = e;
            }
            __syncthreads();
            const double z = geo[4 * a] + (double)k1 * geo[4 * a + 1] + (double)k2 * geo[4 * a + 2];
            const double zf = floor(z);
            const T t = (T)(z - zf);
            int mi = (int)zf - mlo;
            mi = mi < 0 ? 0 : (mi >= R ? R - 1 : mi);
            const T *bk = s_b + c * smax;
            int sub = 0;
            for (int i = 1; i < nsub; ++i) sub += (t >= bk[i]) ? 1 : 0;
            const T *e = E + (mi * nsub + sub) * D1;
            T v = e[D1 - 1];
            for (int k = D1 - 2; k >= 0; --k) v = v * t + e[k];
            const T yk = v - comp;
            const T tk = acc + yk;
            comp = (tk - acc) - yk;
            acc = tk;
            parity ^= 1;
        }
    }
    if (k1 < N && k2 < N) b[(size_t)k2 * N + k1] = acc;
}

// Per-angle interpolant tables for the tiled kernel.  For angle a, bin row
// m in [0, MT) (bin mA_a + m of the angle's window over the whole tile grid)
// and sub-interval s:
//   E[a][m][s][k] = sum_{j < J} p[a][mA_a + m + jlo_a + j] C[a][s][j][k],
// the polynomial (in the offset t within the bin) of the
// weighted sum of the J sinogram samples that reach a pixel whose projection
// falls in that bin and sub-interval; k < D1, padded to 8 with zeros (rows of
// absent sub-intervals are zero).  p is the prefiltered row, zero outside
// [0, M + 2K).  Built once per angle and bin instead of once per (tile,
// angle): a bin row is shared by every tile whose window contains it.  One
// thread per (m, s) row (neighbouring threads write neighbouring rows); the
// sums run over j in increasing order.
template <typename T>
__global__ void __launch_bounds__(256)
k_bp_etab(const T *__restrict__ pf, T *__restrict__ etab, int Mp, int K, int MT,
          const int32_t *__restrict__ ints, const T *__restrict__ coef, int smax, int J, int D1)
{
    constexpr int D1P = 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sC = reinterpret_cast<T *>(smem_raw);  // [smax][J][8] of this angle, zero past D1
    const int a = blockIdx.y, per = smax * J * D1;
    for (int i = threadIdx.x; i < smax * J * D1P; i += blockDim.x) {
        const int k = i % D1P, sj = i / D1P;
        sC[i] = k < D1 ? coef[(size_t)a * per + sj * D1 + k] : T(0);
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MT * smax) return;
    const int m = i / smax, sidx = i - m * smax;
    T e[D1P];
#pragma unroll
    for (int k = 0; k < D1P; ++k) e[k] = T(0);
    if (sidx < ints[4 * a]) {
        const int base = ints[4 * a + 3] + m + ints[4 * a + 1] + K;  // p index of tap 0
        const T *prow = pf + (size_t)a * Mp;
        for (int j = 0; j < J; ++j) {
            const int mi = base + j;
            const T pv = (mi >= 0 && mi < Mp) ? prow[mi] : T(0);
            const T *c = sC + (sidx * J + j) * D1P;
#pragma unroll
            for (int k = 0; k < D1P; ++k) e[k] += pv * c[k];  // (+0 stays +0 past D1)
        }
    }
    // the row as 16-byte stores (rows are 16-byte aligned)
    uint4 *dst = reinterpret_cast<uint4 *>(etab + (size_t)(a * MT + m) * smax * D1P + sidx * D1P);
    const uint4 *src = reinterpret_cast<const uint4 *>(e);
#pragma unroll
    for (int q = 0; q < (int)(D1P * sizeof(T) / 16); ++q) dst[q] = src[q];
}

// Tiled back projection (the default).  A block owns a BP_TX x BP_TY pixel
// tile and one of `groups` contiguous ranges of angles (partial images are
// summed by k_bp_reduce in group order).  Per chunk of CH angles:
//   - thread c: the tile's bin window [mlo, mlo + R) and the split of
//     the tile origin's projection z_t into an integer zi and a fraction;
//     a pixel at offset (d1, d2) in the tile then has z = zi + zl with
//     zl = frac(z_t) + d1 dz1 + d2 dz2 computed in T (|zl| < R);
//   - the window's rows of the angle's table (k_bp_etab) are copied to LDS
//     (16 bytes per thread and step; rows outside the table are zero);
//   - each thread evaluates 8 pixels (rows 4 apart) per angle: one floor,
//     a sub-interval search (branch-free over the SB breakpoints the angle
//     keeps in registers; SB = 0: a loop over them in LDS), one or two
//     16-byte LDS reads, an HN-term Horner scheme (HN >= D1: the
//     coefficients past D1 are the zero padding).
// The windows of a run of BP_WB angles are computed at once (their geometry
// loads wait once per run, not per chunk).  The chunk's angles are summed
// plainly per pixel, then added to a compensated total once per chunk.
// z = i + t with i = floor(z) and t in [0, 1): in FP32 one fract and one
// floor-convert instead of floor, convert and subtract.  The values are the
// same (z - floor(z) is exact) except where z is a tiny negative number and
// z - floor(z) rounds up to 1: fract returns the largest float below 1.
template <typename T>
__device__ __forceinline__ void split_floor(T z, int &i, T &t)
{
    if constexpr (sizeof(T) == 4) {
        t = __builtin_amdgcn_fractf(z);
        asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(z));  // floor and convert in one instruction
    } else {
        const T f = floor(z);
        t = z - f;
        i = (int)f;
    }
}

template <typename T, int HN, int SB>
__global__ void __launch_bounds__(BP_NT, BP_WAVES)
k_bp_tile(const T *__restrict__ etab, T *__restrict__ out, int N, int n, int MT, int groups,
          const double *__restrict__ geo, const int32_t *__restrict__ ints, const T *__restrict__ brk,
          int smax, int rmax, int CH, int LP)
{
    constexpr int NT = BP_NT, D1P = 8, PPT = BP_TX * BP_TY / NT, RSTEP = NT / BP_TX, WB = BP_WB;
    constexpr int V = 16 / sizeof(T);  // elements per 16-byte piece
    // a table row is PR pieces in global memory, of which its HN coefficients
    // fill NPR; in LDS the rows are LP pieces apart (bp_lp: odd where the
    // tables still fit, so that rows at random bins fall on 8 distinct
    // 16-byte positions per 128 bytes; with 32-byte rows, 4 of them, the
    // gathers met twice the bank conflicts)
    constexpr int PR = D1P / V, NPR = (HN + V - 1) / V;
    const int LRS = LP * V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int eang = rmax * smax * LRS;
    // table rows E [CH][rmax][smax][D1P]; for a run of WB angles:
    // breakpoints [WB][smax], (frac(z_t), dz1, dz2) [WB][3] and (g0, R, nsub,
    // zi - mlo) [WB][4], g0 = mlo - mA_a the window's first row in the
    // angle's table
    T *s_E = reinterpret_cast<T *>(smem_raw);
    T *s_b = s_E + (size_t)CH * eang;
    T *s_f = s_b + WB * smax;
    int *s_w = reinterpret_cast<int *>(s_f + WB * 3);
    const int tid = threadIdx.x;
    const int k1a = blockIdx.x * BP_TX, k2a = blockIdx.y * BP_TY;
    const int d1 = tid % BP_TX, d2 = tid / BP_TX;  // rows d2 + RSTEP i
    const int gsz = (n + groups - 1) / groups;
    const int abeg = blockIdx.z * gsz, aend = min(n, abeg + gsz);
    const int rowp = smax * NPR;  // 16-byte pieces copied per bin of a table window
    // the table rows of window entries [c0, c0 + cnt) (angles A + c) to
    // LDS, 16 bytes per thread and step (rows outside [0, MT) are zero):
    // piece i is piece i % NPR of the window's row i / NPR
    auto stage = [&](int A, int c0, int cnt) {
        const uint4 *src = reinterpret_cast<const uint4 *>(etab);
        for (int c = 0; c < cnt; ++c) {
            const int *w = s_w + 4 * (c0 + c);
            const int a = A + c0 + c, tot = w[1] * rowp, g0 = w[0];
            const int lo = max(0, -g0) * rowp, hi = min(w[1], MT - g0) * rowp;
            const int64_t r0 = ((int64_t)a * MT + g0) * smax;  // the window's first row
            uint4 *dst = reinterpret_cast<uint4 *>(s_E + (size_t)c * eang);
            for (int i = tid; i < tot; i += NT) {
                const int r = i / NPR, k = i - r * NPR;
                dst[r * LP + k] = (i >= lo && i < hi) ? src[(r0 + r) * PR + k] : make_uint4(0, 0, 0, 0);
            }
        }
    };
    T acc[PPT], comp[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) acc[i] = comp[i] = T(0);
    for (int A = abeg; A < aend; A += WB) {
        const int cntW = min(WB, aend - A);
        // windows of the run's angles (the previous run's are no longer read)
        if (tid < cntW) {
            const int a = A + tid;
            const double z0 = geo[4 * a], dz1 = geo[4 * a + 1], dz2 = geo[4 * a + 2];
            const double zt = z0 + (double)k1a * dz1 + (double)k2a * dz2;
            const double e1 = (BP_TX - 1) * dz1, e2 = (BP_TY - 1) * dz2;
            const double zmin = zt + fmin(e1, 0.0) + fmin(e2, 0.0);
            const double zmax = zt + fmax(e1, 0.0) + fmax(e2, 0.0);
            const int mlo = (int)floor(zmin) - 1;
            const double zi = floor(zt);
            int *w = s_w + 4 * tid;
            T *f = s_f + 3 * tid;
            w[0] = mlo - ints[4 * a + 3];
            w[1] = min((int)floor(zmax) + 2 - mlo, rmax);
            w[2] = ints[4 * a];
            w[3] = (int)zi - mlo;
            f[0] = (T)(zt - zi);
            f[1] = (T)dz1;
            f[2] = (T)dz2;
        }
        for (int i = tid; i < cntW * smax; i += NT) s_b[i] = brk[(size_t)A * smax + i];
        for (int c0 = 0; c0 < cntW; c0 += CH) {
            const int cnt = min(CH, cntW - c0);
            __syncthreads();  // windows written; the previous chunk's evaluations are done
            stage(A, c0, cnt);
            __syncthreads();
            // the chunk's angles summed plainly per pixel, then added to the
            // compensated total once per chunk
            T csum[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) csum[i] = T(0);
            for (int c = 0; c < cnt; ++c) {
                const int *w = s_w + 4 * (c0 + c);
                const T *f = s_f + 3 * (c0 + c);
                const int R = w[1], nsub = w[2], base = w[3];
                const T zf = f[0], dz1 = f[1], dz2 = f[2];
                const T *bk = s_b + (c0 + c) * smax;
                const T *Ec = s_E + (size_t)c * eang;
                const T zrow = zf + (T)d1 * dz1 + (T)d2 * dz2;
                const T rstep = (T)RSTEP * dz2;
                // value of the angle's interpolant at pixel i, given its row
                // (bin, sub-interval) and offset t in the bin
                auto row = [&](int mi, int sub) { return Ec + (__umul24(mi, smax) + sub) * LRS; };
                auto horner = [&](int i, const T *ev, T u) {
                    T v = ev[HN - 1];
#pragma unroll
                    for (int k = HN - 2; k >= 0; --k) v = v * u + ev[k];
                    csum[i] += v;
                };
                // bin of pixel i in the window; the unsigned minimum keeps it
                // in [0, R) (it is there already up to a rounding of the
                // in-tile position, which the window's one-bin margins absorb)
                auto bin_of = [&](T zl, T &t) {
                    int fl;
                    split_floor(zl, fl, t);
                    return (int)min((unsigned)(base + fl), (unsigned)(R - 1));
                };
                if constexpr (SB > 0) {
                    // branch-free search over the angle's breakpoints held in
                    // registers (SB >= smax; entries at or past nsub are 2,
                    // never passed since t < 1; the first, 0, is not needed)
                    T bb[SB];
#pragma unroll
                    for (int q = 1; q < SB; ++q) bb[q] = q < smax ? bk[q] : T(2);
#pragma unroll
                    for (int i = 0; i < PPT; ++i) {
                        T t;
                        const int mi = bin_of(zrow + (T)i * rstep, t);
                        int sub = 0;
#pragma unroll
                        for (int q = 1; q < SB; ++q) sub += (int)(t >= bb[q]);
                        const T *e = row(mi, sub);
                        T ev[HN];
#pragma unroll
                        for (int k = 0; k < HN; ++k) ev[k] = e[k];
                        horner(i, ev, t);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < PPT; ++i) {
                        T t;
                        const int mi = bin_of(zrow + (T)i * rstep, t);
                        int sub = 0;
                        for (int s2 = 1; s2 < nsub; ++s2) sub += (t >= bk[s2]) ? 1 : 0;
                        const T *e = row(mi, sub);
                        T ev[HN];
#pragma unroll
                        for (int k = 0; k < HN; ++k) ev[k] = e[k];
                        horner(i, ev, t);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const T yk = csum[i] - comp[i];
                const T tk = acc[i] + yk;
                comp[i] = (tk - acc[i]) - yk;
                acc[i] = tk;
            }
        }
        __syncthreads();  // the run's windows are read before the next run writes them
    }
    T *dst = groups > 1 ? out + (size_t)blockIdx.z * N * N : out;
    const int k1 = k1a + d1;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int k2 = k2a + d2 + RSTEP * i;
        if (k1 < N && k2 < N) dst[(size_t)k2 * N + k1] = acc[i];
    }
}

// b = sum over angle groups of the partial images, in group order
template <typename T>
__global__ void __launch_bounds__(256) k_bp_reduce(const T *__restrict__ part, int groups, size_t len,
                                                   T *__restrict__ b)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
        T s = 0;
        for (int g = 0; g < groups; ++g) s += part[(size_t)g * len + i];
        b[i] = s;
    }
}

// Tiled kernel for the plan's Horner length HN (the kernel degree + 1
// rounded up to 4, 6 or 8) and breakpoint registers SB (the most
// sub-intervals of an angle rounded up to 5, 9 or, in FP32, 16; 0: more,
// searched in LDS).  With one detector box generic angles have 5
// sub-intervals at bin width 1 (the fractional parts of the footprint's four
// kinks, and 0) and 9 at bin width 1/2.
static int bp_hn(const gct_plan *p) { return p->bp.D1 <= 4 ? 4 : (p->bp.D1 <= 6 ? 6 : 8); }
static int bp_sb(const gct_plan *p, size_t elem)
{
    const int s = p->bp.smax;
    return s <= 5 ? 5 : (s <= 9 ? 9 : (s <= 16 && elem == 4 ? 16 : 0));
}
int bp_breakpoint_regs(const gct_plan *p, size_t elem) { return bp_sb(p, elem); }
#define GCT_BP_TILE_CASES(CASE)                                                                        \
    switch (bp_hn(p) * 32 + bp_sb(p, sizeof(T))) {                                                    \
    case 4 * 32 + 5: CASE(4, 5); break;                                                               \
    case 4 * 32 + 9: CASE(4, 9); break;                                                               \
    case 4 * 32 + 16: if constexpr (sizeof(T) == 4) CASE(4, 16); break; /* FP32 only */              \
    case 4 * 32 + 0: CASE(4, 0); break;                                                               \
    case 6 * 32 + 5: CASE(6, 5); break;                                                               \
    case 6 * 32 + 9: CASE(6, 9); break;                                                               \
    case 6 * 32 + 16: if constexpr (sizeof(T) == 4) CASE(6, 16); break;                              \
    case 6 * 32 + 0: CASE(6, 0); break;                                                               \
    case 8 * 32 + 5: CASE(8, 5); break;                                                               \
    case 8 * 32 + 9: CASE(8, 9); break;                                                               \
    case 8 * 32 + 16: if constexpr (sizeof(T) == 4) CASE(8, 16); break;                              \
    default: CASE(8, 0); break;                                                                       \
    }
template <typename T>
static const void *bp_tile_fn(const gct_plan *p)
{
    const void *fn = nullptr;
#define GCT_BP_FN(HN_, SB_) fn = reinterpret_cast<const void *>(&k_bp_tile<T, HN_, SB_>)
    GCT_BP_TILE_CASES(GCT_BP_FN)
#undef GCT_BP_FN
    return fn;
}

// Bins of a tile's window and the LDS bytes of the tiled kernel for `ch`
// angles per chunk (table rows; breakpoints and windows of a run of BP_WB
// angles).
static int bp_rmax(const gct_plan *p) { return (int)std::ceil(p->bp.tile_win) + 4; }
// pieces of 16 bytes that a table row's coefficients fill (NPR of k_bp_tile)
static int bp_npr(const gct_plan *p, size_t elem)
{
    const int v = (int)(16 / elem);
    return (bp_hn(p) + v - 1) / v;
}
static size_t bp_tile_lds(const gct_plan *p, size_t elem, int ch, int lp)
{
    return ((size_t)ch * bp_rmax(p) * p->bp.smax * lp * (16 / elem) + (size_t)BP_WB * (p->bp.smax + 3)) * elem +
           (size_t)BP_WB * 4 * sizeof(int);
}
// LDS bytes of the table kernel (one angle's coefficients, padded to 8)
static size_t bp_etab_lds(const gct_plan *p, size_t elem)
{
    return (size_t)p->bp.smax * p->bp.J * 8 * elem;
}

// Launch shape of the tiled kernel for one element size, chosen for
// occupancy.  Angles per chunk: among 8, 4, 2, 1 with tables within 64 KB,
// the one that keeps the most blocks resident per CU
// (hipOccupancyMaxActiveBlocksPerMultiprocessor: registers and LDS), the
// larger on a tie (fewer chunk set-ups).  Angle groups g <= min(32, n / 8)
// minimising ceil(tiles g / resident blocks of the chip) / g: a block's
// work shrinks as 1/g, and a last round of blocks that fills only part of
// the chip leaves CUs idle; the smaller g on a tie (fewer partial images).
template <typename T>
static void bp_configure_t(gct_plan *p, int t)
{
    p->bp_ch[t] = 0;
    p->bp_groups[t] = 1;
    p->bp_lp[t] = 0;
    // beyond the kernels' limits (8 coefficients per table row, 16 taps,
    // one angle's coefficients in LDS)
    if (p->bp.D1 > 8 || p->bp.J > 16 || bp_etab_lds(p, sizeof(T)) > 65536) return;
    const void *fn = bp_tile_fn<T>(p);
    int best_ch = 0, best_nb = 0, best_lp = 0;
    // the odd row stride first; the dense one when only that fits
    const int npr = bp_npr(p, sizeof(T));
    for (int lp : {npr | 1, npr}) {
        for (int ch : {8, 4, 2, 1}) {
            const size_t lds = bp_tile_lds(p, sizeof(T), ch, lp);
            if (lds > 65536) continue;
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, BP_NT, lds) != hipSuccess) nb = 1;
            if (nb > best_nb) {
                best_nb = nb;
                best_ch = ch;
                best_lp = lp;
            }
        }
        if (best_ch > 0) break;
    }
    if (best_ch == 0) return;
    p->bp_lp[t] = best_lp;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1)
        cus = 256;
    const long long tiles = (long long)((p->N + BP_TX - 1) / BP_TX) * ((p->N + BP_TY - 1) / BP_TY);
    const long long slots = (long long)std::max(best_nb, 1) * cus;
    const int gmax = std::max(1, std::min(32, p->n / 8));
    int best_g = 1;
    double best_cost = 1e300;
    for (int g = 1; g <= gmax; ++g) {
        const double cost = (double)((tiles * g + slots - 1) / slots) / g;
        if (cost < best_cost * (1.0 - 1e-12)) {
            best_cost = cost;
            best_g = g;
        }
    }
    p->bp_ch[t] = best_ch;
    p->bp_groups[t] = best_g;
}

void bp_configure(gct_plan *p)
{
    bp_configure_t<float>(p, 0);
    bp_configure_t<double>(p, 1);
    (void)hipGetLastError();  // an occupancy query that failed leaves no error behind
}

int bp_angle_groups(const gct_plan *p, size_t elem) { return p->bp_groups[elem == 4 ? 0 : 1]; }

BPWorkspace bp_workspace(const gct_plan *p, size_t elem)
{
    const int t = elem == 4 ? 0 : 1;
    const bool tiled = p->bp_ch[t] > 0;
    BPWorkspace w;
    size_t o = align256((size_t)p->n * (p->M + 2 * p->K) * elem);
    w.etab = o;
    if (tiled) o += align256((size_t)p->n * p->bp.MT * p->bp.smax * 8 * elem);
    w.part = o;
    if (tiled && p->bp_groups[t] > 1) o += align256((size_t)p->bp_groups[t] * p->N * p->N * elem);
    w.total = o;
    return w;
}

// Tile side, bins per tile window and angles per chunk such that the LDS
// stays within 64 KB: 32 x 32 tiles when they fit, else 16 x 16, else 8 x 8
// (kernels with many sub-intervals: several detector boxes in FP64).
static BPLayout bp_layout(const gct_plan *p, size_t elem)
{
    BPLayout L{16, 0, 1, 0};
    for (int tile : {32, 16, 8}) {
        const int r = (int)std::ceil((tile - 1) * p->bp.span_per_pixel) + 4;
        for (int ch : {16, 8, 4, 2, 1}) {
            const size_t per_coef = (size_t)p->bp.smax * p->bp.J * p->bp.D1;
            const size_t words = 2 * (size_t)r * p->bp.smax * p->bp.D1 + ch * per_coef +
                                 (size_t)ch * (r + p->bp.J) + (size_t)ch * p->bp.smax;
            if (words * elem <= 65536) return BPLayout{tile, r, ch, words * elem};
        }
        L = BPLayout{tile, r, 1, 0};
    }
    L.lds = ~size_t(0);  // does not fit
    return L;
}

size_t bp_lds_bytes(const gct_plan *p, size_t elem) { return bp_layout(p, elem).lds; }

int bp_fallback_tile(const gct_plan *p, size_t elem)
{
    const BPLayout L = bp_layout(p, elem);
    return L.lds <= 65536 ? L.tile : 0;
}

template <typename T>
hipError_t launch_backproject(const gct_plan *p, const T *pf, T *b, T *part, T *etab, hipStream_t s)
{
    const int N = p->N;
    const T *brk_ = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_brk_f32 : p->dev.bp_brk_f64);
    const T *coef_ = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_coef_f32 : p->dev.bp_coef_f64);
    {
        const int t = sizeof(T) == 4 ? 0 : 1;
        const int ch = p->bp_ch[t], rmax = bp_rmax(p);
        if (ch > 0) {
            const int groups = p->bp_groups[t], MT = p->bp.MT, smax = p->bp.smax;
            const double *geo_ = reinterpret_cast<const double *>(p->dev.bp_geo);
            const int32_t *ints_ = reinterpret_cast<const int32_t *>(p->dev.bp_int);
            hipLaunchKernelGGL(k_bp_etab<T>, dim3((unsigned)((MT * smax + 255) / 256), (unsigned)p->n), dim3(256),
                               bp_etab_lds(p, sizeof(T)), s, pf, etab, p->M + 2 * p->K, p->K, MT, ints_, coef_,
                               smax, p->bp.J, p->bp.D1);
            const dim3 grid((N + BP_TX - 1) / BP_TX, (N + BP_TY - 1) / BP_TY, groups);
            T *dst = groups > 1 ? part : b;
            const int lp = p->bp_lp[t];
            const size_t lds = bp_tile_lds(p, sizeof(T), ch, lp);
#define GCT_BP_TILE(HN_, SB_)                                                                             \
    hipLaunchKernelGGL((k_bp_tile<T, HN_, SB_>), grid, dim3(BP_NT), lds, s, (const T *)etab, dst, N, p->n, MT, \
                       groups, geo_, ints_, brk_, smax, rmax, ch, lp)
            GCT_BP_TILE_CASES(GCT_BP_TILE)
#undef GCT_BP_TILE
            if (groups > 1) {
                const size_t len = (size_t)N * N;
                hipLaunchKernelGGL(k_bp_reduce<T>, dim3((unsigned)std::min<size_t>(2048, (len + 255) / 256)),
                                   dim3(256), 0, s, (const T *)part, groups, len, b);
            }
            return hipGetLastError();
        }
    }
    const BPLayout L = bp_layout(p, sizeof(T));
    if (L.lds > 65536) return hipErrorInvalidConfiguration;
    const dim3 grid((N + L.tile - 1) / L.tile, (N + L.tile - 1) / L.tile);
    const T *brk = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_brk_f32 : p->dev.bp_brk_f64);
    const T *coef = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_coef_f32 : p->dev.bp_coef_f64);
    const double *geo = reinterpret_cast<const double *>(p->dev.bp_geo);
    const int32_t *ints = reinterpret_cast<const int32_t *>(p->dev.bp_int);
    if (L.tile == 32)
        hipLaunchKernelGGL((k_backproject<T, 32>), grid, dim3(1024), L.lds, s, pf, b, N, p->n,
                           p->M + 2 * p->K, p->K, geo, ints, brk, coef, p->bp.smax, p->bp.J,
                           p->bp.D1, L.rmax, L.ch);
    else if (L.tile == 8)
        hipLaunchKernelGGL((k_backproject<T, 8>), grid, dim3(64), L.lds, s, pf, b, N, p->n,
                           p->M + 2 * p->K, p->K, geo, ints, brk, coef, p->bp.smax, p->bp.J,
                           p->bp.D1, L.rmax, L.ch);
    else
        hipLaunchKernelGGL((k_backproject<T, 16>), grid, dim3(256), L.lds, s, pf, b, N, p->n,
                           p->M + 2 * p->K, p->K, geo, ints, brk, coef, p->bp.smax, p->bp.J,
                           p->bp.D1, L.rmax, L.ch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward model (Sec. 2; Sec. 4 eq. xray_of_f / eq. blurxray_of_f).
// g[a][m] = sum_k c_k l1 l2 M_[L, M, S](y_m - x_k.u): one thread per
// (angle, bin) walks the image rows (or columns) and visits only the pixels
// whose footprint support contains y_m.  The three-direction footprint is
//   l1 l2 M_[L,M,S](x) = (l1 l2 / L) [Theta(x + L/2) - Theta(x - L/2)],
// Theta(x) = integral_0^x M_[M,S], an odd, bounded function: no cancellation.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T theta_int(const FwdAngle<T> &f, T x)
{
    const T ax = fabs(x);
    const T h1 = (f.M - f.S) * T(0.5), h2 = (f.M + f.S) * T(0.5);
    T r;
    if (ax >= h2) {
        r = T(0.5);
    } else if (ax <= h1) {
        r = ax * f.iM;
    } else {
        const T t = h2 - ax;
        r = T(0.5) - t * t * f.i2MS;
    }
    return x < T(0) ? -r : r;
}

template <typename T>
__device__ __forceinline__ T footprint(const FwdAngle<T> &f, T x)
{
    return f.scale_over_L * (theta_int(f, x + T(0.5) * f.L) - theta_int(f, x - T(0.5) * f.L));
}

// fa holds NB boxes per angle (NB = 0: nb at run time, the detector's
// boxes of Sec. 2; one box of width zeta is the paper's blur); the
// footprint is the sum of the boxes' terms, the support the widest.
template <typename T, int NB>
__global__ void __launch_bounds__(256)
k_forward(const T *__restrict__ c, T *__restrict__ g, int N, int M, double ly,
          const FwdAngle<T> *__restrict__ fa, int nb)
{
    const int a = blockIdx.y;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int nbx = NB > 0 ? NB : nb;
    const FwdAngle<T> *fb = fa + (size_t)a * nbx;
    const FwdAngle<T> f = fb[0];
    const double y = ly * ((double)m - 0.5 * (M - 1));
    const double h = 0.5 * (N - 1);
    double half = (double)f.half;
    for (int b = 1; b < nbx; ++b) half = fmax(half, (double)fb[b].half);
    T acc = 0;
    // walk rows (solve for k1) or columns (solve for k2)
    const double along = f.rows ? f.cx : f.sx;   // coefficient of the solved index
    const double across = f.rows ? f.sx : f.cx;  // coefficient of the walked index
    const double inva = 1.0 / along;
    const double w = half * fabs(inva);
    for (int i = 0; i < N; ++i) {
        const double base = across * ((double)i - h);
        const double ctr = (y - base) * inva + h;  // solved index whose centre projects to y
        int lo = (int)ceil(ctr - w), hi = (int)floor(ctr + w);
        lo = max(lo, 0);
        hi = min(hi, N - 1);
        for (int j = lo; j <= hi; ++j) {
            const T d = (T)(y - base - along * ((double)j - h));
            T v = footprint(f, d);
            for (int b = 1; b < nbx; ++b) v += footprint(fb[b], d);
            const size_t idx = f.rows ? (size_t)i * N + j : (size_t)j * N + i;
            acc += c[idx] * v;
        }
    }
    g[(size_t)a * M + m] = acc;
}

template <typename T>
hipError_t launch_forward(const gct_plan *p, const T *c, T *g, hipStream_t s)
{
    const dim3 grid((p->M + 255) / 256, p->n);
    const FwdAngle<T> *fa =
        reinterpret_cast<const FwdAngle<T> *>(sizeof(T) == 4 ? p->dev.fwd_f32 : p->dev.fwd_f64);
    if (p->fwd_nb == 1) hipLaunchKernelGGL((k_forward<T, 1>), grid, dim3(256), 0, s, c, g, p->N, p->M, p->ly, fa, 1);
    else hipLaunchKernelGGL((k_forward<T, 0>), grid, dim3(256), 0, s, c, g, p->N, p->M, p->ly, fa, p->fwd_nb);
    return hipGetLastError();
}

template hipError_t launch_prefilter<float>(const gct_plan *, const float *, float *, hipStream_t);
template hipError_t launch_prefilter<double>(const gct_plan *, const double *, double *, hipStream_t);
template hipError_t launch_backproject<float>(const gct_plan *, const float *, float *, float *, float *,
                                              hipStream_t);
template hipError_t launch_backproject<double>(const gct_plan *, const double *, double *, double *, double *,
                                               hipStream_t);
template hipError_t launch_forward<float>(const gct_plan *, const float *, float *, hipStream_t);
template hipError_t launch_forward<double>(const gct_plan *, const double *, double *, hipStream_t);

}  // namespace gct
