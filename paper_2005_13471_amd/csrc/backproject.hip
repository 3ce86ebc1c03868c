// Sinogram interpolation, exact-adjoint back projection and the forward
// model (Sec. 2, Sec. 4, Sec. 5).
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
// B-spline basis of the interpolated sinogram.  kappa is evaluated from the
// per-angle sub-interval polynomials built exactly on the host.
//
// One 16 x 16 pixel tile per block.  Angle tables are staged through LDS
// in chunks; each lane then locates its sub-interval and accumulates the
// J weighted bins.
// ---------------------------------------------------------------------------
constexpr int BP_CHUNK = 8;

template <typename T>
__global__ void __launch_bounds__(256)
k_backproject(const T *__restrict__ pf, T *__restrict__ b, int N, int n, int Mp, int K,
              const double *__restrict__ geo, const int32_t *__restrict__ ints,
              const T *__restrict__ brk, const T *__restrict__ coef, int smax, int J, int D1)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per_coef = smax * J * D1;
    T *s_coef = reinterpret_cast<T *>(smem_raw);                 // [CHUNK][smax][J][D1]
    T *s_brk = s_coef + BP_CHUNK * per_coef;                     // [CHUNK][smax]
    double *s_geo = reinterpret_cast<double *>(s_brk + BP_CHUNK * smax + (BP_CHUNK * smax) % 2);
    int32_t *s_int = reinterpret_cast<int32_t *>(s_geo + BP_CHUNK * 4);

    const int k1 = blockIdx.x * 16 + (threadIdx.x & 15);
    const int k2 = blockIdx.y * 16 + (threadIdx.x >> 4);
    T acc = 0, comp = 0;
    for (int a0 = 0; a0 < n; a0 += BP_CHUNK) {
        const int cnt = min(BP_CHUNK, n - a0);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * per_coef; i += blockDim.x)
            s_coef[i] = coef[(size_t)a0 * per_coef + i];
        for (int i = threadIdx.x; i < cnt * smax; i += blockDim.x) s_brk[i] = brk[(size_t)a0 * smax + i];
        for (int i = threadIdx.x; i < cnt * 4; i += blockDim.x) {
            s_geo[i] = geo[(size_t)a0 * 4 + i];
            s_int[i] = ints[(size_t)a0 * 4 + i];
        }
        __syncthreads();
        for (int c = 0; c < cnt; ++c) {
            const double z = s_geo[4 * c] + (double)k1 * s_geo[4 * c + 1] + (double)k2 * s_geo[4 * c + 2];
            const double zf = floor(z);
            const T t = (T)(z - zf);
            const int m0 = (int)zf;
            const int nsub = s_int[4 * c], jlo = s_int[4 * c + 1];
            const T *bk = s_brk + c * smax;
            int sub = 0;
            for (int i = 1; i < nsub; ++i) sub += (t >= bk[i]) ? 1 : 0;
            const T u = t - bk[sub];
            const T *cf = s_coef + (size_t)c * per_coef + (size_t)sub * J * D1;
            const T *prow = pf + (size_t)(a0 + c) * Mp;
            T sum = 0;
            for (int j = 0; j < J; ++j) {
                T w = cf[j * D1 + D1 - 1];
                for (int d = D1 - 2; d >= 0; --d) w = w * u + cf[j * D1 + d];
                const int mi = m0 + jlo + j + K;
                const T pv = (mi >= 0 && mi < Mp) ? prow[mi] : T(0);
                sum += pv * w;
            }
            const T yk = sum - comp;
            const T tk = acc + yk;
            comp = (tk - acc) - yk;
            acc = tk;
        }
    }
    if (k1 < N && k2 < N) b[(size_t)k2 * N + k1] = acc;
}

size_t bp_lds_bytes(const gct_plan *p, size_t elem)
{
    const size_t per_coef = (size_t)p->bp.smax * p->bp.J * p->bp.D1;
    size_t t = (BP_CHUNK * per_coef + BP_CHUNK * p->bp.smax + 1) * elem;
    t = (t + 7) & ~size_t(7);
    return t + BP_CHUNK * 4 * sizeof(double) + BP_CHUNK * 4 * sizeof(int32_t);
}

template <typename T>
hipError_t launch_backproject(const gct_plan *p, const T *pf, T *b, hipStream_t s)
{
    const int N = p->N;
    const dim3 grid((N + 15) / 16, (N + 15) / 16);
    const T *brk = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_brk_f32 : p->dev.bp_brk_f64);
    const T *coef = reinterpret_cast<const T *>(sizeof(T) == 4 ? p->dev.bp_coef_f32 : p->dev.bp_coef_f64);
    hipLaunchKernelGGL(k_backproject<T>, grid, dim3(256), bp_lds_bytes(p, sizeof(T)), s, pf, b, N,
                       p->n, p->M + 2 * p->K, p->K, reinterpret_cast<const double *>(p->dev.bp_geo),
                       reinterpret_cast<const int32_t *>(p->dev.bp_int), brk, coef, p->bp.smax,
                       p->bp.J, p->bp.D1);
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
