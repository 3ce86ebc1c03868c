// Gram filtering (Sec. 4, closing remark): H^T H is Toeplitz-block-Toeplitz,
// so y = H^T H c is the zero-padded linear convolution of the N x N
// coefficients with the (2N-1)^2 Gram filter.  It is evaluated exactly (up
// to rounding) through the P x P circulant embedding, P >= 2N-1 a power of
// two or (1536, 3072) three times one: y = IFFT2(Ghat . FFT2(c_padded))[0:N,
// 0:N], with Ghat real and even because G[k] = G[-k].
//
// Three passes, each a block-local FFT (fft_common.h):
//   rows:    pairs of image rows -> one complex FFT -> two real-row spectra,
//            written transposed as W1[w1][k2], w1 in [0, P/2];
//   columns: per w1, FFT along k2 (N nonzero of P), times Ghat[w1][.],
//            inverse FFT, keep k2 < N -> W2[w1][k2];
//   rows:    pairs of Hermitian row spectra -> one complex inverse FFT ->
//            two real output rows, keep k1 < N.
// The 1/P^2 normalisation is folded into Ghat.  One block of P/E threads
// owns one transform.
#include <algorithm>
#include <mutex>

#include "fft_passes.h"

namespace gct {

// One transform per block, P/E threads; E is the plan's choice for the
// apply passes (gct_plan_autotune), fft_elems(P) for the spectrum.
template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
k_rows_fwd(const T *__restrict__ src, C2<T> *__restrict__ W1, int N, const C2<T> *__restrict__ tw)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int rp = xcd_swizzle(blockIdx.x, gridDim.x);
    // data first, then the twiddles: their latencies overlap
    C2<T> v[E];
    rows_fwd_load<T, PC, E>(2 * rp, src, N, nullptr, T(0), v);
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    rows_fwd_regs<T, PC, E>(2 * rp, v, W1, N, x, tws);
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
k_cols(const C2<T> *__restrict__ W1, C2<T> *__restrict__ W2, const T *__restrict__ Ghat, int N,
       const C2<T> *__restrict__ tw)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    C2<T> v[E];
    T gs[E];
    cols_load<T, PC, E>(blockIdx.x, W1, Ghat, N, v, gs);
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    cols_regs<T, PC, E>(blockIdx.x, v, gs, W2, N, x, tws);
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
k_rows_inv(const C2<T> *__restrict__ W2, T *__restrict__ y, int N, const C2<T> *__restrict__ tw)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int rp = xcd_swizzle(blockIdx.x, gridDim.x);
    C2<T> v[E];
    rows_inv_load<T, PC, E>(2 * rp, W2, N, v);
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    fft_passes<T, E, P, 1, true, true>(v, x, threadIdx.x, tws);
    (void)rows_inv_store<T, PC, E>(2 * rp, v, y, N, nullptr);
}

template <typename T, int PC>
__global__ void __launch_bounds__(256)
k_spec_rows(const T *__restrict__ G, C2<T> *__restrict__ R, int N, const C2<T> *__restrict__ tw)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / fft_elems(P)>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    body_spec_rows<T, PC, fft_elems(P)>(xcd_swizzle(blockIdx.x, gridDim.x), G, R, N, x, tws);
}

template <typename T, int PC>
__global__ void __launch_bounds__(256)
k_spec_cols(const C2<T> *__restrict__ R, T *__restrict__ Ghat, const C2<T> *__restrict__ tw,
            T scale)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / fft_elems(P)>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    body_spec_cols<T, PC, fft_elems(P)>(blockIdx.x, R, Ghat, x, tws, scale);
}

// ---------------------------------------------------------------------------
// Fused CG iteration (single slice), in the Chronopoulos-Gear arrangement:
// one product w = A r and one reduction point per iteration.  Launch i:
//   rows_fwd: every block reduces the previous launch's partial dots
//     gamma = r.r and delta = r.w (fixed order) and, unless ||r||^2 = gamma
//     meets the stopping rule, takes
//       beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
//     (beta = 0, alpha = gamma / delta for the first update), then on its own
//     two rows p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//     and transforms the new r;
//   cols: unchanged;
//   rows_inv: w = A r on its rows and the partial dots r.r, r.w.
// In exact arithmetic these are the textbook CG iterates (s = A p; the
// denominator is p.Ap).  With the state's steepest-descent flag every update
// takes beta = 0 (p = r, s = w = A r, alpha = r.r / r.A r: the paper's
// solver, Sec. 6.2).  All blocks compute the same scalars; block 0 alone
// records them, in the slots of the other parity.
// ---------------------------------------------------------------------------
// (sum part[0..np), sum part[np..2np)) in a fixed order, for a block of NT
// threads: thread t adds entries t, t + NT, ... in increasing order.  The
// first KP of them are loaded by part_load (clamped addresses, so the loads
// can be issued before anything else), the rest, if any, here.
template <int NT, int KP>
__device__ __forceinline__ void part_load(const double *part, int np, double (&pg)[KP], double (&pd)[KP])
{
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const int i = min((int)threadIdx.x + j * NT, np - 1);
        pg[j] = part[i];
        pd[j] = part[np + i];
    }
}

template <int NT, int KP>
__device__ __forceinline__ void dot_pair(const double *part, int np, const double (&pg)[KP],
                                         const double (&pd)[KP], double *red, double &g, double &d)
{
    g = 0.0;
    d = 0.0;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        if ((int)threadIdx.x + j * NT < np) {
            g += pg[j];
            d += pd[j];
        }
    }
    for (int i = threadIdx.x + KP * NT; i < np; i += NT) {
        g += part[i];
        d += part[np + i];
    }
    block_sum2<NT>(g, d, red);
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
k_cgf_rows_fwd(T *__restrict__ x, T *__restrict__ r, T *__restrict__ p, T *__restrict__ sv,
               const T *__restrict__ w, C2<T> *__restrict__ W1, int N, const C2<T> *__restrict__ tw,
               CGState *st, const double *__restrict__ part, int np, int par)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *xs = reinterpret_cast<C2<T> *>(smem_raw);
    double *red = reinterpret_cast<double *>(smem_raw);
    const int rp = xcd_swizzle(blockIdx.x, gridDim.x);
    const int ra = 2 * rp;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const int64_t stat = st->stat[par], pend = st->pend[par];
    // the previous launch's partial dots and this thread's elements of the
    // five vectors (in range whatever the state), issued together with the
    // state words so that all their latencies overlap
    // (entries q >= E/2 are at t + G q >= P/2 >= N: never loaded, zero in
    // the transform)
    constexpr int G = P / E, KP = E / 4 + 1, H = E / 2;
    double pg[KP], pd[KP];
    part_load<G, KP>(part, np, pg, pd);
    T lr[H][2], lw[H][2], lp[H][2], ls[H][2], lx[H][2];
#pragma unroll
    for (int q = 0; q < H; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = threadIdx.x + G * q, row = ra + h;
            const bool ok = n < N && row < N;
            const size_t i = ok ? (size_t)row * N + n : 0;
            lr[q][h] = ok ? r[i] : T(0);
            lw[q][h] = ok ? w[i] : T(0);
            lp[q][h] = ok ? p[i] : T(0);
            ls[q][h] = ok ? sv[i] : T(0);
            lx[q][h] = ok ? x[i] : T(0);
        }
    if (stat != CG_RUNNING) return;
    if (pend) {
        // twiddles to LDS behind the data area (the reduction below uses
        // its start): their latency overlaps the loads above
        const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(xs + fft_data_elems<T>(P), tw);
        double g, dl;
        dot_pair<G, KP>(part, np, pg, pd, red, g, dl);
        const int64_t u = st->k;  // updates so far: g = ||r_u||^2
        if (!(g == g)) {
            if (lead) st->stat[par ^ 1] = st->status = CG_BREAKDOWN;
            return;
        }
        if (g <= st->thr2) {
            if (lead) {
                st->ring[u % CG_RING] = g;
                st->kring = u;
                st->rr = g;
                st->stat[par ^ 1] = st->status = CG_CONVERGED;
            }
            return;
        }
        double alpha, beta;
        const bool sd = st->sd != 0;  // steepest descent: no conjugation
        if (pend == 1 || sd) {
            beta = 0.0;
            alpha = g / dl;
        } else {
            beta = g / st->gam[par ^ 1];
            alpha = g / (dl - beta * g / st->alp[par ^ 1]);
        }
        if (!(alpha > 0.0) || !(alpha < INFINITY)) {  // p.Ap <= 0 or non-finite
            if (lead) st->stat[par ^ 1] = st->status = CG_BREAKDOWN;
            return;
        }
        if (lead) {
            st->ring[u % CG_RING] = g;
            st->kring = u;
            st->rr = g;
            st->k = u + 1;
            st->gam[par] = g;
            st->alp[par] = alpha;
            st->alpha = alpha;
            st->beta = beta;
            st->pend[par ^ 1] = 2;
            st->stat[par ^ 1] = CG_RUNNING;
        }
        const T al = (T)alpha, be = (T)beta;
        const bool first = pend == 1 || sd;  // p = r, s = w (no direction carried over)
        // thread t owns columns t + G q of the two rows: the same elements
        // the transform takes, so the new r goes to it in registers
        C2<T> v[E];
#pragma unroll
        for (int q = H; q < E; ++q) v[q] = {T(0), T(0)};
#pragma unroll
        for (int q = 0; q < H; ++q) {
            T rv[2] = {T(0), T(0)};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int n = threadIdx.x + G * q, row = ra + h;
                if (n >= N || row >= N) continue;
                const size_t i = (size_t)row * N + n;
                const T pi = first ? lr[q][h] : lr[q][h] + be * lp[q][h];
                const T si = first ? lw[q][h] : lw[q][h] + be * ls[q][h];
                p[i] = pi;
                sv[i] = si;
                x[i] = lx[q][h] + al * pi;
                rv[h] = lr[q][h] - al * si;
                r[i] = rv[h];
            }
            v[q] = {rv[0], rv[1]};
        }
        __syncthreads();  // the reduction's LDS reads are done before the transform writes
        rows_fwd_regs<T, PC, E>(ra, v, W1, N, xs, tws);
        return;
    } else if (lead) {
        st->pend[par ^ 1] = 1;  // first launch: transform r_0 only
        st->stat[par ^ 1] = CG_RUNNING;
    }
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(xs + fft_data_elems<T>(P), tw);
    __syncthreads();
    body_rows_fwd<T, PC, E>(ra, r, W1, N, xs, tws, nullptr, T(0));
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
k_cgf_cols(const C2<T> *__restrict__ W1, C2<T> *__restrict__ W2, const T *__restrict__ Ghat, int N,
           const C2<T> *__restrict__ tw, const CGState *st, int par)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    // the column's loads go out with the state word's (in range either way)
    const int64_t stat = st->stat[par ^ 1];
    C2<T> v[E];
    T gs[E];
    cols_load<T, PC, E>(blockIdx.x, W1, Ghat, N, v, gs);
    if (stat != CG_RUNNING) return;
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    cols_regs<T, PC, E>(blockIdx.x, v, gs, W2, N, x, tws);
}

template <typename T, int PC, int E>
__global__ void __launch_bounds__(256)
k_cgf_rows_inv(const C2<T> *__restrict__ W2, T *__restrict__ w, const T *__restrict__ r, int N,
               const C2<T> *__restrict__ tw, const CGState *st, double *__restrict__ part, int np, int par)
{
    constexpr int P = fft_size(PC);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T> *x = reinterpret_cast<C2<T> *>(smem_raw);
    const int rp = xcd_swizzle(blockIdx.x, gridDim.x);
    const int ra = 2 * rp, rb = ra + 1;
    constexpr int G = P / E;
    const int64_t stat = st->stat[par ^ 1];  // tested after the loads below are issued
    // this thread's entries of r, loaded ahead of the transform so that
    // their latency overlaps it
    // (clamped in-range addresses; entries past N are never used)
    // (q < E/2 only: t + G q >= P/2 >= N beyond)
    T lr[E / 2][2];
    const size_t oa = (size_t)ra * N, ob = rb < N ? oa + N : oa;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
        const int nc = min((int)threadIdx.x + G * q, N - 1);
        lr[q][0] = r[oa + nc];
        lr[q][1] = r[ob + nc];
    }
    C2<T> v[E];
    rows_inv_load<T, PC, E>(ra, W2, N, v);
    if (stat != CG_RUNNING) return;
    const C2<T> *tws = stage_twiddles<T, twiddles_in_lds<T>(P), P / 2, P / E>(x + fft_data_elems<T>(P), tw);
    __syncthreads();
    fft_passes<T, E, P, 1, true, true>(v, x, threadIdx.x, tws);
    double g = 0.0, dl = 0.0;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
        const int n = threadIdx.x + G * q;
        if (n >= N) continue;
        const size_t ia = (size_t)ra * N + n;
        w[ia] = v[q].x;
        const double ra_ = (double)lr[q][0];
        g += ra_ * ra_;
        dl += ra_ * (double)v[q].x;
        if (rb < N) {
            const size_t ib = ia + N;
            w[ib] = v[q].y;
            const double rb_ = (double)lr[q][1];
            g += rb_ * rb_;
            dl += rb_ * (double)v[q].y;
        }
    }
    __syncthreads();  // the transform's LDS reads are done before red is written
    block_sum2<G>(g, dl, reinterpret_cast<double *>(smem_raw));
    if (threadIdx.x == 0) {
        part[rp] = g;
        part[np + rp] = dl;
    }
}

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
struct FftCfg {
    int threads;   // P / E
    size_t lds;    // bytes of dynamic LDS
};

template <typename T>
static FftCfg fft_cfg(int pc)
{
    const int P = fft_size(pc);
    return FftCfg{P / fft_elems(P), fft_lds_bytes<T>(P, fft_elems(P))};
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
#define GCT_LAUNCH_FFT(kern, T, pc, cfg, grid, s, ...)                                        \
    do {                                                                                       \
        const dim3 blk_(cfg.threads);                                                          \
        switch (pc) {                                                                        \
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
        case 12: hipLaunchKernelGGL((kern<T, 12>), grid, blk_, cfg.lds, s, __VA_ARGS__); break; \
        case 41: hipLaunchKernelGGL((kern<T, 41>), grid, blk_, cfg.lds, s, __VA_ARGS__); break; \
        default: hipLaunchKernelGGL((kern<T, 42>), grid, blk_, cfg.lds, s, __VA_ARGS__); break; \
        }                                                                                      \
    } while (0)

// Elements per thread the apply passes can take for a length-P transform:
// fft_elems(P) always; for P = 512 also 4, for P = 1024 also 8 and 4, for
// P = 2048 also 8; for P = 3 * 2^k (1536, 3072) 24 and 12 (at most 256
// threads per transform).
bool apply_e_ok(int pc, int E)
{
    const int P = fft_size(pc);
    if (E == fft_elems(P)) return true;
    if (P == 512) return E == 4;
    if (P == 1024) return E == 8 || E == 4;
    if (P == 2048) return E == 8;
    if (P % 3 == 0) return (E == 12 || E == 24) && P / E <= 256;
    return false;
}

#define GCT_ACASE(kern, T, LG, E, grid, lds, s, ...) \
    hipLaunchKernelGGL((kern<T, LG, E>), grid, dim3(fft_size(LG) / E), lds, s, __VA_ARGS__)

#define GCT_LAUNCH_FFTE(kern, T, pc, E, grid, lds, s, ...)                              \
    do {                                                                                  \
        switch (pc) {                                                                   \
        case 2: GCT_ACASE(kern, T, 2, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 3: GCT_ACASE(kern, T, 3, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 4: GCT_ACASE(kern, T, 4, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 5: GCT_ACASE(kern, T, 5, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 6: GCT_ACASE(kern, T, 6, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 7: GCT_ACASE(kern, T, 7, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 8: GCT_ACASE(kern, T, 8, 4, grid, lds, s, __VA_ARGS__); break;               \
        case 9:                                                                           \
            if (E == 4) GCT_ACASE(kern, T, 9, 4, grid, lds, s, __VA_ARGS__);              \
            else GCT_ACASE(kern, T, 9, 8, grid, lds, s, __VA_ARGS__);                     \
            break;                                                                        \
        case 10:                                                                          \
            if (E == 4) GCT_ACASE(kern, T, 10, 4, grid, lds, s, __VA_ARGS__);             \
            else if (E == 8) GCT_ACASE(kern, T, 10, 8, grid, lds, s, __VA_ARGS__);        \
            else GCT_ACASE(kern, T, 10, 16, grid, lds, s, __VA_ARGS__);                   \
            break;                                                                        \
        case 11:                                                                          \
            if (E == 8) GCT_ACASE(kern, T, 11, 8, grid, lds, s, __VA_ARGS__);             \
            else GCT_ACASE(kern, T, 11, 16, grid, lds, s, __VA_ARGS__);                   \
            break;                                                                        \
        case 12: GCT_ACASE(kern, T, 12, 16, grid, lds, s, __VA_ARGS__); break;            \
        GCT_MIXED_CASES(GCT_ACASE, kern, T, E, grid, lds, s, __VA_ARGS__)                 \
        }                                                                                 \
    } while (0)

// The three passes of one apply.
template <typename T>
hipError_t launch_gram_apply(const gct_plan *p, const T *Ghat, const T *c, T *y, void *ws, hipStream_t s)
{
    const int N = p->N, P = p->P, pc = p->pc;
    const int t = sizeof(T) == 4 ? 0 : 1, E = p->fft_e[t], Ec = p->fft_ec[t];
    const size_t lds = fft_lds_bytes<T>(P, E), ldsc = fft_lds_bytes<T>(P, Ec);
    const size_t w1 = align256((size_t)(P / 2 + 1) * N * 2 * sizeof(T));
    C2<T> *W1 = reinterpret_cast<C2<T> *>(ws);
    C2<T> *W2 = reinterpret_cast<C2<T> *>(reinterpret_cast<char *>(ws) + w1);
    const C2<T> *tw = twiddles<T>(p);
    const dim3 rgrid((N + 1) / 2), cgrid(P / 2 + 1);
    GCT_LAUNCH_FFTE(k_rows_fwd, T, pc, E, rgrid, lds, s, c, W1, N, tw);
    GCT_LAUNCH_FFTE(k_cols, T, pc, Ec, cgrid, ldsc, s, W1, W2, Ghat, N, tw);
    GCT_LAUNCH_FFTE(k_rows_inv, T, pc, E, rgrid, lds, s, W2, y, N, tw);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cgf_iteration(const gct_plan *p, const T *Ghat, T *x, T *r, T *pv, T *sv, T *w, void *ws,
                                double *part, CGState *st, int par, hipStream_t s)
{
    const int N = p->N, P = p->P, pc = p->pc;
    const int t = sizeof(T) == 4 ? 0 : 1, E = p->cg_e[t], Ec = p->cg_ec[t];
    const size_t lds = fft_lds_bytes<T>(P, E), ldsc = fft_lds_bytes<T>(P, Ec);
    const size_t w1 = align256((size_t)(P / 2 + 1) * N * 2 * sizeof(T));
    C2<T> *W1 = reinterpret_cast<C2<T> *>(ws);
    C2<T> *W2 = reinterpret_cast<C2<T> *>(reinterpret_cast<char *>(ws) + w1);
    const C2<T> *tw = twiddles<T>(p);
    const int np = (N + 1) / 2;
    const dim3 rgrid(np), cgrid(P / 2 + 1);
    GCT_LAUNCH_FFTE(k_cgf_rows_fwd, T, pc, E, rgrid, lds, s, x, r, pv, sv, (const T *)w, W1, N, tw, st,
                    (const double *)part, np, par);
    GCT_LAUNCH_FFTE(k_cgf_cols, T, pc, Ec, cgrid, ldsc, s, (const C2<T> *)W1, W2, Ghat, N, tw,
                    (const CGState *)st, par);
    GCT_LAUNCH_FFTE(k_cgf_rows_inv, T, pc, E, rgrid, lds, s, (const C2<T> *)W2, w, (const T *)r, N, tw,
                    (const CGState *)st, part, np, par);
    return hipGetLastError();
}

template hipError_t launch_cgf_iteration<float>(const gct_plan *, const float *, float *, float *, float *,
                                                float *, float *, void *, double *, CGState *, int, hipStream_t);
template hipError_t launch_cgf_iteration<double>(const gct_plan *, const double *, double *, double *,
                                                 double *, double *, double *, void *, double *, CGState *,
                                                 int, hipStream_t);

template <typename T>
hipError_t launch_gram_spectrum(const gct_plan *p, const T *G, T *Ghat, void *ws, hipStream_t s)
{
    const int N = p->N, P = p->P, pc = p->pc;
    const FftCfg c = fft_cfg<T>(pc);
    C2<T> *R = reinterpret_cast<C2<T> *>(ws);
    const C2<T> *tw = twiddles<T>(p);
    GCT_LAUNCH_FFT(k_spec_rows, T, pc, c, dim3(P / 2), s, G, R, N, tw);
    const T scale = T(1.0 / ((double)P * (double)P));
    GCT_LAUNCH_FFT(k_spec_cols, T, pc, c, dim3(P / 2 + 1), s, R, Ghat, tw, scale);
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

}  // namespace gct

// ---------------------------------------------------------------------------
// Gram filtering without a workspace argument (gct_gram_apply_static), for
// callers that cannot allocate device memory.  The transposed scratch
// arrays W1, W2 of the three passes live in `scratch`, a file-scope device
// array: every GPU the library runs on holds its own copy until the process
// ends.  Host code never names the array in a launch; it uses the address
// hipGetSymbolAddress returns for the current device, fetched once per
// device.  Every used entry of W1 and W2 is written before it is read, so
// nothing needs clearing between calls; calls that overlap on one GPU share
// the array and race.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t STATIC_SCRATCH_BYTES = size_t(24) << 20;  // 24 MiB
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (the current device).
int static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return gct::fail(GCT_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return gct::check_hip(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return gct::fail(GCT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GCT_OK;
}

}  // namespace

extern "C" int gct_gram_apply_static(const gct_plan *p, gct_dtype dt, const void *Ghat, const void *c,
                                     void *y, void *stream)
{
    using namespace gct;
    if (!p) return fail(GCT_EINVAL, "plan is NULL");
    if (dt != GCT_F32 && dt != GCT_F64) return fail(GCT_EINVAL, "bad dtype");
    if (!Ghat || !c || !y) return fail(GCT_EINVAL, "NULL buffer");
    if (c == y) return fail(GCT_EINVAL, "y must not alias c");
    const size_t need = apply_ws_bytes(p, dt == GCT_F32 ? 4 : 8);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(GCT_EINVAL, "gram_apply_static: this plan needs " + std::to_string(need) +
                                    " bytes of scratch, more than the static array's " +
                                    std::to_string(STATIC_SCRATCH_BYTES) +
                                    "; use gct_gram_apply with a workspace");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return check_hip(e, "hipGetDevice");
    if (dev != p->device) return fail(GCT_EINVAL, "the current device is not the plan's device");
    void *ws = nullptr;
    const int rc = static_scratch(dev, &ws);
    if (rc != GCT_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = dt == GCT_F32 ? launch_gram_apply<float>(p, (const float *)Ghat, (const float *)c, (float *)y, ws, s)
                      : launch_gram_apply<double>(p, (const double *)Ghat, (const double *)c, (double *)y, ws, s);
    return check_hip(e, "gram_apply_static launch");
}

