// Gram filter construction (Sec. 4).
//
// G[k] = sum over angles of A_theta(k1 l1 cos + k2 l2 sin), where A_theta is
// the autocorrelation of the projected pixel: the centred univariate box
// spline with directions {l1|c|, l1|c|, l2|s|, l2|s|} (Sec. 4, four-direction
// spline), plus {zeta, zeta} with detector blur (six-direction spline), times
// (l1 l2)^2.  Because the footprint is even, its autocorrelation equals its
// self-convolution.
//
// Evaluation in FP32 without cancellation.  With T_w = M_[w,w] (triangle of
// half-width w, height 1/w) and {L >= M >= S} the sorted directions,
// A = T_L * T_M * T_S.  Writing psi_w(y) = (w - |y|)_+^3 / (6 w^2) and
// chi_S(y) = (S - |y|)_+^5 / (120 S^2), one has exactly
//   A(x)   = T_L(x) + [rho(x + L) - 2 rho(x) + rho(x - L)] / L^2,
//   rho(y) = psi_M(y) + (S^2/12) T_M(y)
//            + [chi_S(y + M) - 2 chi_S(y) + chi_S(y - M)] / M^2.
// (Derivation: T_w = w^-2 * second difference of |x|/2 with step w;
// (|x|/2) * T_w = |x|/2 + psi_w; (|x|^3/12) * T_S = |x|^3/12 + |x| S^2/24 +
// chi_S; then collect the smooth parts.)  Every term is bounded by about
// M/6 and no large intermediate cancels, unlike the truncated-power sum,
// which loses all digits in FP32 at near-axis angles where one direction is
// tiny.  A zero direction drops out (its constants are 0).
//
// Tap offsets are formed in FP64 (k1 cx + k2 sx reaches ~1.5e3 at N = 1024
// while the spline needs them to ~1e-7) and rounded once.  The sum over
// angles is compensated (Kahan).  G[k] = G[-k] holds exactly (the footprint
// is even), so half the taps are evaluated and mirrored; when the plan's
// angle set and pixels give G the eight symmetries of the square (gram_d4),
// only the octant 0 <= k2 <= k1 is evaluated and each tap is written to its
// eight images.
#include <cmath>

#include "gct_internal.h"

namespace gct {

template <typename T>
__device__ __forceinline__ T pos1(T t) { return t > T(0) ? t : T(0); }

template <typename T>
__device__ __forceinline__ T chi5(const GramAngle<T> &g, T y)
{
    const T t = pos1(g.S - fabs(y));
    const T t2 = t * t;
    return t2 * t2 * t * g.c120S;
}

template <typename T>
__device__ __forceinline__ T rho(const GramAngle<T> &g, T y, bool blur)
{
    const T t = pos1(g.M - fabs(y));
    T r = t * t * t * g.c6M;
    if (blur) {
        r += g.s12 * t * g.iM2;
        r += (chi5(g, y + g.M) - T(2) * chi5(g, y) + chi5(g, y - g.M)) * g.iM2;
    }
    return r;
}

template <typename T>
__device__ __forceinline__ T gram_A(const GramAngle<T> &g, T x, bool blur)
{
    const T ax = fabs(x);
    if (ax >= g.half) return T(0);
    const T tl = pos1(g.L - ax) * g.iL2;
    const T r = rho(g, x + g.L, blur) - T(2) * rho(g, x, blur) + rho(g, x - g.L, blur);
    return g.scale * (tl + r * g.iL2);
}

// One square tile of taps per block (side below), covering only taps with
// k2 > 0 or (k2 = 0, k1 >= 0); each such tap also writes its mirror -k (G
// is even).  With d4 the tiles cover the octant instead: tile (bx, by),
// by <= bx, holds taps (bx TS + tx, by TS + ty), and the taps with
// k2 <= k1 < N write all eight images.
//
// Angular windows.  Tap k projects to k1 l1 cos + k2 l2 sin = rho cos(theta -
// phi) with (rho, phi) the polar form of (k1 l1, k2 l2), so A_theta(k) can be
// nonzero only where |cos(theta - phi)| < h / rho (h = support half-width):
// theta within asin(h / rho) of phi + pi/2, mod pi.  Over the tile (polar
// angles [phi_lo, phi_hi], distance >= rho_min from the origin) every
// contributing angle lies in [phi_lo + pi/2 - d, phi_hi + pi/2 + d] mod pi,
// d = asin(h_max / rho_min): at most two runs of the angles sorted by
// theta mod pi, found by binary search.  Inside a run the exact per-angle
// test on the tile's projected interval still applies, so the window only
// has to contain every contributing angle.
//
// Work split.  The window is taken in chunks of 256 angles: thread t loads
// angle t of the chunk and tests it against the tile, and the angles that
// pass are packed in order into LDS (wave ballots, so the order is fixed;
// per-angle loads straight from the tables were a chain of two dependent
// scalar loads per angle).  SPLIT (one slice, 8 x 8 taps per block): the
// block's NW waves (4 or 8) each hold the tile's 64 taps and take every
// NW-th packed angle, so the tiles at the origin, which every angle reaches
// and which set the kernel's duration, cost 1/NW of the angles per wave;
// the NW compensated partial sums are added in wave order at the end.  Not
// SPLIT (batches, 16 x 16 taps per block, many more tiles than CUs): every
// thread owns one tap and takes every packed angle.
__device__ __forceinline__ int lower_idx(const double *th, int n, double v)
{
    int lo = 0, hi = n;  // first index with th >= v
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (th[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The same search by a whole wave (v uniform): 64 evenly spaced probes
// locate the segment, then one probe per element of it; two rounds of loads
// instead of log2(n) dependent ones.  Every lane returns the index.
__device__ __forceinline__ int lower_idx_wave(const double *th, int n, double v)
{
    const int lane = threadIdx.x & 63;
    const int step = (n + 63) / 64;
    if (step > 64) return lower_idx(th, n, v);
    const int p = min(n - 1, lane * step + step - 1);
    const int seg = __popcll(__ballot(th[p] < v));  // probes below v: the answer is past them
    const int base = seg * step;
    const int i = base + lane;
    const bool below = lane < step && i < n && th[i] < v;
    return min(n, base + __popcll(__ballot(below)));
}

// Tile (bx, by) of the octant's triangle of T tiles a side, by <= bx, from
// its index k in [0, T (T + 1) / 2) (rows of the triangle in order).
__device__ __forceinline__ void octant_tile(int k, int T, int &bx, int &by)
{
    by = 0;
    while (k >= T - by) {
        k -= T - by;
        ++by;
    }
    bx = by + k;
}

template <typename T, bool SPLIT, int NW>
__device__ __forceinline__ void body_gram_tile(int bx, int by, T *__restrict__ G, int N, int n,
                                               const GramAngle<T> *__restrict__ ga,
                                               const int32_t *__restrict__ ord, const double *__restrict__ th,
                                               double hmax, double l1, double l2, bool d4)
{
    constexpr int TS = SPLIT ? GRAM_TILE_SPLIT : GRAM_TILE;
    __shared__ GramAngle<T> sg[256];
    __shared__ int wcnt[NW];
    __shared__ T racc[NW][64], rcomp[NW][64];
    const int W = 2 * N - 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tap = SPLIT ? lane : tid;  // SPLIT: every wave holds the tile's 64 taps
    const int tx = tap % TS, ty = tap / TS;
    const int k1a = d4 ? bx * TS : bx * TS - (N - 1);  // first tap column of the tile
    const int k2a = by * TS;                          // first tap row (>= 0)
    const int k1 = k1a + tx, k2 = k2a + ty;
    const bool live = d4 ? (k1 <= N - 1 && k2 <= k1) : (k1 <= N - 1 && k2 <= N - 1 && (k2 > 0 || k1 >= 0));
    const double ka = k1a, kb = k1a + TS - 1, la = k2a, lb = k2a + TS - 1;
    // the tile's runs of sorted angles (the same in every thread)
    int run_lo[2] = {0, 0}, run_hi[2] = {n, 0};
    const double x0 = ka * l1, x1 = kb * l1, y0 = la * l2, y1 = lb * l2;  // y0 >= 0
    const double dx = x0 > 0.0 ? x0 : (x1 < 0.0 ? -x1 : 0.0);
    const double dy = y0;
    const double rmin = sqrt(dx * dx + dy * dy);
    if (rmin > hmax * 1.000001 + 1e-9) {
        const double f00 = atan2(y0, x0), f01 = atan2(y1, x0), f10 = atan2(y0, x1), f11 = atan2(y1, x1);
        const double flo = fmin(fmin(f00, f01), fmin(f10, f11));
        const double fhi = fmax(fmax(f00, f01), fmax(f10, f11));
        const double d = asin(hmax / rmin) + 1e-9;
        const double a0 = flo + 0.5 * M_PI - d, b0 = fhi + 0.5 * M_PI + d;
        if (b0 - a0 < M_PI) {
            double a = fmod(a0, M_PI);
            if (a < 0.0) a += M_PI;
            const double b = a + (b0 - a0);
            run_lo[0] = lower_idx_wave(th, n, a);
            if (b <= M_PI) {
                run_hi[0] = lower_idx_wave(th, n, b);
            } else {
                run_hi[0] = n;
                run_hi[1] = lower_idx_wave(th, n, b - M_PI);
            }
        }
    }
    const double dk1 = k1, dk2 = k2;
    T acc = 0, comp = 0;
    for (int run = 0; run < 2; ++run)
        for (int j0 = run_lo[run]; j0 < run_hi[run]; j0 += 256) {
            const int cnt = min(256, run_hi[run] - j0);
            GramAngle<T> g;
            bool hit = false;
            if (tid < cnt) {  // (the first 256 threads)
                g = ga[ord[j0 + tid]];
                // projected interval of the tile (extreme corners)
                const double p1 = ka * g.cx, p2 = kb * g.cx, q1 = la * g.sx, q2 = lb * g.sx;
                const double dmin = fmin(p1, p2) + fmin(q1, q2), dmax = fmax(p1, p2) + fmax(q1, q2);
                hit = dmax > -(double)g.half && dmin < (double)g.half;
            }
            const unsigned long long mask = __ballot(hit);
            __syncthreads();  // the previous chunk's readers are done with sg and wcnt
            if (lane == 0) wcnt[wave] = __popcll(mask);
            __syncthreads();
            int off = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                off += w < wave ? wcnt[w] : 0;
                total += wcnt[w];
            }
            if (hit) sg[off + __popcll(mask & ((1ull << lane) - 1ull))] = g;
            __syncthreads();
            for (int jj = SPLIT ? wave : 0; jj < total; jj += SPLIT ? NW : 1) {
                const GramAngle<T> &h = sg[jj];
                const T dd = (T)(dk1 * h.cx + dk2 * h.sx);
                const T v = h.S > T(0) ? gram_A(h, dd, true) : gram_A(h, dd, false);
                const T yk = v - comp;
                const T tk = acc + yk;
                comp = (tk - acc) - yk;
                acc = tk;
            }
        }
    // tap (a, b) of value v at row b, column a; with d4 its eight images
    auto put = [&](T v) {
        G[(size_t)(k2 + N - 1) * W + (k1 + N - 1)] = v;
        G[(size_t)(N - 1 - k2) * W + (N - 1 - k1)] = v;
        if (d4) {
            G[(size_t)(k2 + N - 1) * W + (N - 1 - k1)] = v;
            G[(size_t)(N - 1 - k2) * W + (k1 + N - 1)] = v;
            G[(size_t)(k1 + N - 1) * W + (k2 + N - 1)] = v;
            G[(size_t)(N - 1 - k1) * W + (N - 1 - k2)] = v;
            G[(size_t)(k1 + N - 1) * W + (N - 1 - k2)] = v;
            G[(size_t)(N - 1 - k1) * W + (k2 + N - 1)] = v;
        }
    };
    if (!SPLIT) {
        if (live) put(acc);
        return;
    }
    racc[wave][lane] = acc;
    rcomp[wave][lane] = comp;
    __syncthreads();
    if (wave == 0 && live) {
        // compensated sum of the NW partial sums (value acc - comp each), in order
        T s = 0, c = 0;
#pragma unroll
        for (int w = 0; w < 2 * NW; ++w) {
            const T v = (w & 1) ? -rcomp[w >> 1][lane] : racc[w >> 1][lane];
            const T yk = v - c;
            const T tk = s + yk;
            c = (tk - s) - yk;
            s = tk;
        }
        put(s);
    }
}

template <typename T, int NW>
__global__ void __launch_bounds__(64 * NW)
k_gram_build(T *__restrict__ G, int N, int n, const GramAngle<T> *__restrict__ ga, const int32_t *__restrict__ ord,
             const double *__restrict__ th, double hmax, double l1, double l2, int d4)
{
    int bx = blockIdx.x, by = blockIdx.y;  // d4: a one-dimensional grid over the octant's tiles
    if (d4) octant_tile(blockIdx.x, (N + GRAM_TILE_SPLIT - 1) / GRAM_TILE_SPLIT, bx, by);
    body_gram_tile<T, true, NW>(bx, by, G, N, n, ga, ord, th, hmax, l1, l2, d4 != 0);
}

// Batched: block b covers tile map[b].y of slice map[b].x.
template <typename T>
__global__ void __launch_bounds__(256)
kb_gram_build(const int2 *__restrict__ map, const BatchSlice *__restrict__ sl, T *__restrict__ G)
{
    const int2 m = map[blockIdx.x];
    const BatchSlice &d = sl[m.x];
    int bx, by;
    if (d.gd4) {
        octant_tile(m.y, (d.N + GRAM_TILE - 1) / GRAM_TILE, bx, by);
    } else {
        const int tiles_x = (2 * d.N - 1 + GRAM_TILE - 1) / GRAM_TILE;
        bx = m.y % tiles_x;
        by = m.y / tiles_x;
    }
    body_gram_tile<T, false, 4>(bx, by, G + d.gram, d.N, d.n, reinterpret_cast<const GramAngle<T> *>(d.ga), d.gord,
                             d.gth, d.ghmax, d.l1, d.l2, d.gd4 != 0);
}

template <typename T>
hipError_t launch_gram_build(const gct_plan *p, T *G, hipStream_t s)
{
    const int W = 2 * p->N - 1, TN = (p->N + GRAM_TILE_SPLIT - 1) / GRAM_TILE_SPLIT;
    const dim3 grid = p->gram_d4 ? dim3(TN * (TN + 1) / 2) : dim3((W + GRAM_TILE_SPLIT - 1) / GRAM_TILE_SPLIT, TN);
    // Waves per block: the tiles at the origin, which every angle reaches,
    // take n / NW angles per wave; the far tiles take few, and larger blocks
    // leave more of their waves idle and fewer blocks resident.  8 waves when
    // the tiles are few against the angles (at most 6 n), else 4.  Measured
    // on MI355X (ms, 4 / 8 / 16 waves): 512^2 / 720 angles, octant 0.069 /
    // 0.043 / 0.056, half plane 0.073 / 0.084 / 0.144; 1024^2 / 1440 octant
    // 0.132 / 0.100 / 0.178; 2048^2 / 1800 octant 0.23 / 0.44 / 0.84.
    const bool wide = (long long)grid.x * grid.y <= 6LL * p->n;
    const GramAngle<T> *ga =
        reinterpret_cast<const GramAngle<T> *>(sizeof(T) == 4 ? p->dev.gram_f32 : p->dev.gram_f64);
    const int32_t *ord = reinterpret_cast<const int32_t *>(p->dev.gram_ord);
    const double *th = reinterpret_cast<const double *>(p->dev.gram_th);
    if (wide)
        hipLaunchKernelGGL((k_gram_build<T, 8>), grid, dim3(512), 0, s, G, p->N, p->gram_n, ga, ord, th, p->gram_hmax,
                           p->lx1, p->lx2, p->gram_d4);
    else
        hipLaunchKernelGGL((k_gram_build<T, 4>), grid, dim3(256), 0, s, G, p->N, p->gram_n, ga, ord, th, p->gram_hmax,
                           p->lx1, p->lx2, p->gram_d4);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_gram_build(const int2 *map, int nblocks, const BatchSlice *sl, T *G,
                                   hipStream_t s)
{
    if (nblocks > 0) hipLaunchKernelGGL(kb_gram_build<T>, dim3(nblocks), dim3(256), 0, s, map, sl, G);
    return hipGetLastError();
}

template hipError_t launch_batch_gram_build<float>(const int2 *, int, const BatchSlice *, float *,
                                                   hipStream_t);
template hipError_t launch_batch_gram_build<double>(const int2 *, int, const BatchSlice *, double *,
                                                    hipStream_t);
template hipError_t launch_gram_build<float>(const gct_plan *, float *, hipStream_t);
template hipError_t launch_gram_build<double>(const gct_plan *, double *, hipStream_t);

}  // namespace gct
