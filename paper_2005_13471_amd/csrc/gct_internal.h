// Internal declarations shared by the host plan code and the HIP kernels of
// libgramct.  Not part of the public interface (include/gramct.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gramct.h"

namespace gct {

// ---------------------------------------------------------------------------
// Per-angle tables, built on the host in FP64 and copied to the device.
// ---------------------------------------------------------------------------

// Gram filter (Sec. 4): at each angle the autocorrelated projected pixel is
// the centred box spline A = T_L * T_M * T_S (T_w = M_[w,w], a triangle of
// half-width w and unit integral) with {L >= M >= S} the sorted directions
// {l1|c|, l2|s|, zeta}, times (l1 l2)^2.  Positions use FP64 (cx, sx).
template <typename T>
struct GramAngle {
    double cx, sx;    // l1 cos, l2 sin: tap (k1, k2) projects to k1 cx + k2 sx
    T L, M, S;        // sorted directions
    T iL2;            // 1 / L^2
    T iM2;            // 1 / M^2      (0 if M == 0)
    T c6M;            // 1 / (6 M^2)  (0 if M == 0)
    T s12;            // S^2 / 12
    T c120S;          // 1 / (120 S^2) (0 if S == 0)
    T scale;          // (l1 l2)^2
    T half;           // support half-width L + M + S
};

// Forward projection (Sec. 4 eq. blurxray_of_f): the blurred footprint is
// l1 l2 M_[L, M, S] with {L >= M >= S} = sorted {l1|c|, l2|s|, zeta}.
template <typename T>
struct FwdAngle {
    double cx, sx;    // l1 cos, l2 sin (FP64 positions)
    T L, M, S;
    T iL;             // 1/L
    T iM;             // 1/M (0 if M == 0)
    T i2MS;           // 1/(2 M S) (0 if S == 0)
    T scale_over_L;   // l1 l2 / L
    T half;           // (L + M + S)/2
    int32_t rows;     // 1: iterate over image rows (|l1 c| >= |l2 s|), 0: over columns
    int32_t pad;
};

// Back projection (Sec. 5).  For a pixel whose centre projects to the
// fractional bin index z = z0 + k1 dz1 + k2 dz2, write z = m0 + t with
// m0 = floor(z), t in [0,1).  Its contribution at this angle is
//   sum_j p[m0 + j] kappa(j - t),  j = jlo .. jlo + J - 1,
// where kappa = l1 l2 M_{Xi / lambda_y}, Xi = {l1|c|, l2|s|, zeta,
// lambda_y x (d+1)}.  On each sub-interval [brk[s], brk[s+1]) of t the
// weights kappa(j - t) are polynomials in u = t - brk[s] with coefficients
// coef[s][j][0..D] (the host tables; the device tables hold them re-expanded
// in powers of t).
struct BPAngleHost {
    double z0, dz1, dz2;
    int32_t nsub, jlo, degree;
};

// Table layout sizes for a plan (padded maxima over all angles).
struct BPDims {
    int32_t smax;   // sub-intervals per angle (padded)
    int32_t J;      // weights per pixel and angle
    int32_t D1;     // polynomial coefficients per weight (degree + 1)
    double span_per_pixel;  // max over angles of (l1|c| + l2|s|) / lambda_y: bins per pixel step
    double tile_win;        // max over angles of (BP_TX-1)|dz1| + (BP_TY-1)|dz2|: bins a tile spans
    int32_t MT;             // bin rows of the per-angle interpolant tables (every tile window)
};

// Pixel tile of the back-projection kernel (columns x rows), its threads
// per block, the minimum resident waves per SIMD it is compiled for, and the
// angles whose bin windows it computes at once.
constexpr int BP_TX = 64, BP_TY = 32, BP_NT = 256, BP_WAVES = 5, BP_WB = 64;
// Gram build: taps per tile side (one block of 4 waves per tile): batched
// builds 16, the single-slice build 8 with the block's waves splitting the
// angles
constexpr int GRAM_TILE = 16, GRAM_TILE_SPLIT = 8;

struct DeviceTables {
    void *gram_f32 = nullptr, *gram_f64 = nullptr;    // GramAngle<T>[n]
    void *fwd_f32 = nullptr, *fwd_f64 = nullptr;      // FwdAngle<T>[n]
    void *bp_geo = nullptr;                           // double[n][4]: z0, dz1, dz2, 0
    void *bp_int = nullptr;                           // int32[n][4]: nsub, jlo, degree, 0
    void *bp_brk_f32 = nullptr, *bp_brk_f64 = nullptr;  // T[n][smax]
    void *bp_coef_f32 = nullptr, *bp_coef_f64 = nullptr;  // T[n][smax][J][D1]
    void *tw_f32 = nullptr, *tw_f64 = nullptr;        // complex twiddles e^{-2 pi i k / P}, k < P/2
    void *q_f32 = nullptr, *q_f64 = nullptr;          // correction filter q[-K..K]
    void *deg = nullptr;                              // int32[n]: B-spline degree per angle
    void *gram_ord = nullptr;  // int32[n]: angle indices sorted by theta mod pi
    void *gram_th = nullptr;   // double[n]: theta mod pi in that order
};

// Device-resident CG state (cg.hip, batch.hip).
constexpr int CG_RING = 64;
enum : int64_t { CG_RUNNING = 0, CG_CONVERGED = 1, CG_BREAKDOWN = 2 };

struct CGState {
    double rr, bb, rr0, pAp, alpha, beta, thr2, pad;
    int64_t k, status, sd, fb;  // sd = 1: steepest descent (every update takes beta = 0);
                                // fb = 1: the start vector was replaced by zero
    double ring[CG_RING];  // ||r_k||^2 at ring[k % CG_RING]
    // fused single-slice iteration (parity slots, see gram_apply.hip):
    // gamma = ||r||^2 and alpha of the last update, "updates may start" (1:
    // first, 2: later) and the device-side status; a kernel reads the slots
    // of its parity and writes the others, so its blocks never race
    double gam[2], alp[2];
    int64_t pend[2], stat[2];
    int64_t kring;  // last index written to ring
};

// One slice of a batch (device descriptor).  Offsets are in elements of the
// packed arrays: image arrays (N^2 per slice), Gram filters ((2N-1)^2),
// spectra ((P/2+1) P reals) and Gram-filtering scratch ((P/2+1) N complex).
struct BatchSlice {
    int32_t N, pc, n, nrow;   // pc: transform size code (fft_size); nrow = ceil(N/2) row pairs
    int64_t img, gram, spec, w;
    int64_t rpart;              // first row-pair partial of this slice
    const void *ga;             // GramAngle<T> table of the slice's plan
    const void *tw;             // twiddles of the slice's plan
    const int32_t *gord;        // angles sorted by theta mod pi (Gram build)
    const double *gth;
    double ghmax;               // largest support half-width of A_theta
    double l1, l2;              // pixel sides
    int32_t gd4;                // the plan's gram_d4
};

// Key of a captured chunk of CG iterations.
// (the right-hand side is not part of it: the iterations read only the
// workspace vectors, x and the spectrum, so solves of many right-hand sides
// reuse one graph)
struct CGGraphKey {
    const void *Ghat;
    void *x, *ws;
    int elem, chunk;
    bool operator==(const CGGraphKey &o) const
    {
        return Ghat == o.Ghat && x == o.x && ws == o.ws && elem == o.elem && chunk == o.chunk;
    }
};

struct CGGraph {
    CGGraphKey key;
    hipGraphExec_t exec;
};

}  // namespace gct

struct gct_plan {
    int32_t N, n, M, K;
    double lx1, lx2, ly, zeta;
    int32_t P, pc;  // transform size and its code (fft_size(pc) == P)
    // Gram-filter table entries (angle, term of the detector's
    // autocorrelation; one term per angle for zero or one box) and
    // footprint boxes per angle
    int32_t gram_n = 0, fwd_nb = 1;
    double gram_hmax;  // largest support half-width of A_theta over the angles
    int gram_d4;       // G has the square's eight symmetries (square pixels, angle set
                       // closed under theta -> theta + pi/2 and theta -> -theta, mod pi)
    // elements per thread of the transforms, [F32, F64]: the row passes and
    // the column pass of an apply, and the same for the fused CG passes
    int32_t fft_e[2], fft_ec[2];
    int32_t cg_e[2], cg_ec[2];
    gct::BPDims bp;
    // launch shape of the tiled back projection, [F32, F64] (bp_configure):
    // angles per chunk (0: the tiled kernel does not apply), angle groups and
    // the LDS row stride of its tables in 16-byte pieces
    int32_t bp_ch[2], bp_groups[2], bp_lp[2];
    gct::DeviceTables dev;
    int64_t dev_bytes = 0;  // bytes of the device tables
    int device;
    // cached CG iteration graphs and the stream they are captured on
    std::vector<gct::CGGraph> cg_graphs;
    hipStream_t capture_stream = nullptr;
    // pinned host copy of the solver state and the event of its copy
    gct::CGState *cg_pin = nullptr;
    hipEvent_t cg_ev = nullptr;
};

namespace gct {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int check_hip(hipError_t e, const char *what);

// ---------------------------------------------------------------------------
bool apply_e_ok(int pc, int E);

// One fused CG iteration of the single-slice solver (gram_apply.hip): the
// update from the previous dots + forward rows of r, columns, inverse rows
// (w = A r) with the partial dots r.r and r.w.  par = launch parity.
template <typename T>
hipError_t launch_cgf_iteration(const gct_plan *p, const T *Ghat, T *x, T *r, T *pv, T *sv, T *w, void *ws,
                                double *part, CGState *st, int par, hipStream_t s);

// Kernel launchers (defined in the .hip files), templated on float/double.
// Each returns hipSuccess or the launch error.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_gram_build(const gct_plan *p, T *G, hipStream_t s);

template <typename T>
hipError_t launch_gram_spectrum(const gct_plan *p, const T *G, T *Ghat, void *ws, hipStream_t s);

template <typename T>
hipError_t launch_gram_apply(const gct_plan *p, const T *Ghat, const T *c, T *y, void *ws,
                             hipStream_t s);

template <typename T>
hipError_t launch_prefilter(const gct_plan *p, const T *g, T *out, hipStream_t s);

template <typename T>
hipError_t launch_backproject(const gct_plan *p, const T *prefiltered, T *b, T *partial, T *etab, hipStream_t s);
int bp_angle_groups(const gct_plan *p, size_t elem);
// Back-projection workspace: the prefiltered sinogram at offset 0, then (the
// tiled kernel) the per-angle interpolant tables at `etab`, then (several
// angle groups) one partial image per group at `part`; byte offsets.
struct BPWorkspace {
    size_t etab, part, total;
};
BPWorkspace bp_workspace(const gct_plan *p, size_t elem);
// Tile side of the per-angle back-projection kernel (taken when the tiled
// kernel's tables do not fit, bp_ch == 0), or 0 when its LDS does not fit.
int bp_fallback_tile(const gct_plan *p, size_t elem);
// Breakpoints the tiled back-projection kernel holds in registers per angle
// (5, 9 or 16; 0: searched in LDS).
int bp_breakpoint_regs(const gct_plan *p, size_t elem);

// Default elements per thread of the row passes and of the column pass for a
// transform of size P (what the autotuner picks on MI355X at P = 1024: the
// row passes fastest with 256 threads per transform, the column pass with
// 128; elsewhere the largest tile, 256 threads at most per transform).
inline void default_pass_elems(int P, int &rows, int &cols)
{
    rows = cols = P % 3 == 0 ? 24 : (P >= 1024 ? 16 : (P == 512 ? 8 : 4));
    if (P == 1024) {
        rows = 4;
        cols = 8;
    }
}

// Transform size of a plan: the smallest P >= 2N - 1 among powers of two and
// (from 1536 up) three times a power of two; its size code (log2 P, or 32 +
// log2(P / 3)).  Below 1536 points the passes are latency-bound and the
// power-of-two kernels, though longer, run as fast or faster (measured at
// N = 384: 768 points 14.8 us per apply, 1024 points 14.3 us); at N = 600
// and 768, 1536 points take 26.7 and 28.5 us against 31.6 and 33.5 us at
// 2048.
inline void choose_fft_size(int N, int &P, int &code)
{
    P = 4;
    code = 2;
    while (P < 2 * N - 1) {
        P <<= 1;
        ++code;
    }
    int P3 = 1536, c3 = 41;
    while (P3 < 2 * N - 1) {
        P3 <<= 1;
        ++c3;
    }
    if (P3 < P) {
        P = P3;
        code = c3;
    }
}
void bp_configure(gct_plan *p);

template <typename T>
hipError_t launch_forward(const gct_plan *p, const T *c, T *g, hipStream_t s);

// Workspace sizing helpers.
size_t apply_ws_bytes(const gct_plan *p, size_t elem);
size_t spectrum_ws_bytes(const gct_plan *p, size_t elem);

// method: 0 = conjugate gradients, 1 = steepest descent (same fused passes
// with beta = 0)
template <typename T>
int cg_solve(const gct_plan *p, const T *Ghat, const T *b, T *x, int use_x0, double rtol,
             int max_iter, int check_every, double *hist, gct_cg_result *res, void *ws,
             hipStream_t s, int method = 0);
size_t cg_ws_bytes(const gct_plan *p, size_t elem);
template <typename T>
int plan_autotune(gct_plan *p, const T *Ghat, void *ws, int reps, int32_t *chosen, hipStream_t s);

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace gct
