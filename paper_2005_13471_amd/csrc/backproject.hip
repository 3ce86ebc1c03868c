// Sinogram interpolation, exact-adjoint back projection and the forward
// model (Sec. 2, Sec. 4, Sec. 5).
#include <cmath>

#include "gct_internal.h"

namespace gct {

// ---------------------------------------------------------------------------
// Correction filter (Sec. 5, eq. correction filter).  One thread per output
// element p[a][m + K], m in [-K, M-1+K]; rows whose B-spline degree is 0 or 1
// are copied (q = delta), degree-2 rows are filtered with the 2K+1 taps.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_prefilter(const T *__restrict__ g, T *__restrict__ out, int n, int M, int K,
            const T *__restrict__ q, const int32_t *__restrict__ deg)
{
    const int Mp = M + 2 * K;
    const int a = blockIdx.y;
    const int mo = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n || mo >= Mp) return;
    const int m = mo - K;
    const T *row = g + (size_t)a * M;
    T acc = 0;
    if (deg[a] == 2) {
        const int jlo = max(-K, m - (M - 1)), jhi = min(K, m);
        for (int j = jlo; j <= jhi; ++j) acc += q[j + K] * row[m - j];
    } else if (m >= 0 && m < M) {
        acc = row[m];
    }
    out[(size_t)a * Mp + mo] = acc;
}

template <typename T>
hipError_t launch_prefilter(const gct_plan *p, const T *g, T *out, hipStream_t s)
{
    const int Mp = p->M + 2 * p->K;
    const dim3 grid((Mp + 255) / 256, p->n);
    const T *q = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.q_f32 : p->dev.q_f64);
    hipLaunchKernelGGL(k_prefilter<T>, grid, dim3(256), 0, s, g, out, p->n, p->M, p->K, q,
                       reinterpret_cast<const int32_t *>(p->dev.deg));
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
// in u = t - brk[s] with coefficients C[s][j][.] (built exactly on the host),
// so the whole angle's contribution is the piecewise polynomial
//   S(z) = sum_k u^k E[m0][s][k],  E[m][s][k] = sum_j p[m + jlo + j] C[s][j][k],
// m0 = floor(z).  A block owns a TILE x TILE pixel tile; per angle it forms E
// for the few bins the tile projects onto (in LDS), then every pixel finds
// its (m0, s) and evaluates one polynomial.  FP64 is used only for z.
// ---------------------------------------------------------------------------
template <typename T, int TILE>
__global__ void __launch_bounds__(TILE * TILE)
k_backproject(const T *__restrict__ pf, T *__restrict__ b, int N, int n, int Mp, int K,
              const double *__restrict__ geo, const int32_t *__restrict__ ints,
              const T *__restrict__ brk, const T *__restrict__ coef, int smax, int J, int D1,
              int rmax)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per_coef = smax * J * D1;
    T *s_E = reinterpret_cast<T *>(smem_raw);   // [rmax][smax][D1]
    T *s_C = s_E + (size_t)rmax * smax * D1;    // [smax][J][D1]
    T *s_p = s_C + per_coef;                    // [rmax + J]
    T *s_b = s_p + rmax + J;                    // [smax]
    const int tid = threadIdx.x;
    const int k1a = blockIdx.x * TILE, k2a = blockIdx.y * TILE;
    const int k1 = k1a + tid % TILE, k2 = k2a + tid / TILE;
    const double kx0 = k1a, kx1 = k1a + TILE - 1, ky0 = k2a, ky1 = k2a + TILE - 1;
    T acc = 0, comp = 0;
    for (int a = 0; a < n; ++a) {
        const double z0 = geo[4 * a], dz1 = geo[4 * a + 1], dz2 = geo[4 * a + 2];
        const int nsub = ints[4 * a], jlo = ints[4 * a + 1];
        // bin range of the tile (with one bin of margin against rounding)
        const double e1 = kx0 * dz1, e2 = kx1 * dz1, f1 = ky0 * dz2, f2 = ky1 * dz2;
        const double zmin = z0 + fmin(e1, e2) + fmin(f1, f2);
        const double zmax = z0 + fmax(e1, e2) + fmax(f1, f2);
        const int mlo = (int)floor(zmin) - 1;
        const int R = min((int)floor(zmax) + 1 - mlo + 1, rmax);
        __syncthreads();  // previous angle done with s_E / s_C / s_p
        for (int i = tid; i < nsub * J * D1; i += TILE * TILE) s_C[i] = coef[(size_t)a * per_coef + i];
        for (int i = tid; i < nsub; i += TILE * TILE) s_b[i] = brk[(size_t)a * smax + i];
        for (int i = tid; i < R + J - 1; i += TILE * TILE) {
            const int mi = mlo + jlo + i + K;
            s_p[i] = (mi >= 0 && mi < Mp) ? pf[(size_t)a * Mp + mi] : T(0);
        }
        __syncthreads();
        const int nE = R * nsub * D1;
        for (int i = tid; i < nE; i += TILE * TILE) {
            const int k = i % D1, rest = i / D1;
            const int sidx = rest % nsub, mi = rest / nsub;
            const T *cf = s_C + sidx * J * D1 + k;
            const T *pp = s_p + mi;
            T e = 0;
            for (int j = 0; j < J; ++j) e += pp[j] * cf[j * D1];
            s_E[i] = e;
        }
        __syncthreads();
        const double z = z0 + (double)k1 * dz1 + (double)k2 * dz2;
        const double zf = floor(z);
        const T t = (T)(z - zf);
        int mi = (int)zf - mlo;
        mi = mi < 0 ? 0 : (mi >= R ? R - 1 : mi);
        int sub = 0;
        for (int i = 1; i < nsub; ++i) sub += (t >= s_b[i]) ? 1 : 0;
        const T u = t - s_b[sub];
        const T *e = s_E + (mi * nsub + sub) * D1;
        T v = e[D1 - 1];
        for (int k = D1 - 2; k >= 0; --k) v = v * u + e[k];
        const T yk = v - comp;
        const T tk = acc + yk;
        comp = (tk - acc) - yk;
        acc = tk;
    }
    if (k1 < N && k2 < N) b[(size_t)k2 * N + k1] = acc;
}

// Tile side and LDS size: 32 x 32 when the per-angle tables fit in 64 KB,
// else 16 x 16.
static int bp_tile(const gct_plan *p, size_t elem, size_t *lds, int *rmax)
{
    for (int tile : {32, 16}) {
        const int r = (int)std::ceil((tile - 1) * p->bp.span_per_pixel) + 4;
        const size_t words = (size_t)r * p->bp.smax * p->bp.D1 + (size_t)p->bp.smax * p->bp.J * p->bp.D1 +
                             r + p->bp.J + p->bp.smax;
        const size_t bytes = words * elem;
        if (bytes <= 65536 || tile == 16) {
            *lds = bytes;
            *rmax = r;
            return tile;
        }
    }
    return 16;
}

size_t bp_lds_bytes(const gct_plan *p, size_t elem)
{
    size_t lds;
    int r;
    bp_tile(p, elem, &lds, &r);
    return lds;
}

template <typename T>
hipError_t launch_backproject(const gct_plan *p, const T *pf, T *b, hipStream_t s)
{
    const int N = p->N;
    size_t lds;
    int rmax;
    const int tile = bp_tile(p, sizeof(T), &lds, &rmax);
    if (lds > 65536) return hipErrorInvalidConfiguration;
    const dim3 grid((N + tile - 1) / tile, (N + tile - 1) / tile);
    const T *brk = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_brk_f32 : p->dev.bp_brk_f64);
    const T *coef = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_coef_f32 : p->dev.bp_coef_f64);
    const double *geo = reinterpret_cast<const double *>(p->dev.bp_geo);
    const int32_t *ints = reinterpret_cast<const int32_t *>(p->dev.bp_int);
    if (tile == 32)
        hipLaunchKernelGGL((k_backproject<T, 32>), grid, dim3(1024), lds, s, pf, b, N, p->n,
                           p->M + 2 * p->K, p->K, geo, ints, brk, coef, p->bp.smax, p->bp.J,
                           p->bp.D1, rmax);
    else
        hipLaunchKernelGGL((k_backproject<T, 16>), grid, dim3(256), lds, s, pf, b, N, p->n,
                           p->M + 2 * p->K, p->K, geo, ints, brk, coef, p->bp.smax, p->bp.J,
                           p->bp.D1, rmax);
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

template <typename T>
__global__ void __launch_bounds__(256)
k_forward(const T *__restrict__ c, T *__restrict__ g, int N, int M, double ly,
          const FwdAngle<T> *__restrict__ fa)
{
    const int a = blockIdx.y;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const FwdAngle<T> f = fa[a];
    const double y = ly * ((double)m - 0.5 * (M - 1));
    const double h = 0.5 * (N - 1);
    const double half = (double)f.half;
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
            const T v = footprint(f, d);
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
    hipLaunchKernelGGL(k_forward<T>, grid, dim3(256), 0, s, c, g, p->N, p->M, p->ly, fa);
    return hipGetLastError();
}

template hipError_t launch_prefilter<float>(const gct_plan *, const float *, float *, hipStream_t);
template hipError_t launch_prefilter<double>(const gct_plan *, const double *, double *, hipStream_t);
template hipError_t launch_backproject<float>(const gct_plan *, const float *, float *, hipStream_t);
template hipError_t launch_backproject<double>(const gct_plan *, const double *, double *,
                                               hipStream_t);
template hipError_t launch_forward<float>(const gct_plan *, const float *, float *, hipStream_t);
template hipError_t launch_forward<double>(const gct_plan *, const double *, double *, hipStream_t);

}  // namespace gct
