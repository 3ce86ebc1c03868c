// Host side of libgramct: geometry validation, per-angle tables built in
// FP64, and the C-ABI entry points of include/gramct.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gramct.h"
#include "../../include/gramct_host.h"
#include "gct_internal.h"

namespace gct {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GCT_OK;
    return fail(GCT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Exact piecewise polynomials for centred univariate box splines.
//
// A box spline with directions w_1..w_r (Sec. 3, eq. boxconv) is the
// convolution of the unit-integral boxes M_w = (1/w) 1_[-w/2, w/2].  It is
// built by repeated convolution, smallest direction first: convolving f with
// M_w gives (F(x + w/2) - F(x - w/2)) / w, F the antiderivative of f.
// Starting from the narrowest box means every later difference spans a
// width at least as large as the features of F, so nothing cancels badly
// even when one direction is tiny (near-axis angles).  Each piece stores
// its polynomial in the local variable (x - left knot).
// ---------------------------------------------------------------------------
constexpr int PP_MAXC = 10;
using Coef = std::array<double, PP_MAXC>;

struct PPoly {
    std::vector<double> x;  // knots, size pieces + 1
    std::vector<Coef> c;    // per piece, coefficients of (x - x_i)^k
    int deg = 0;
};

// b(u) = a(u + d): repeated synthetic division.
static Coef taylor_shift(const Coef &a, int deg, double d)
{
    Coef b = a;
    for (int i = 0; i < deg; ++i)
        for (int j = deg - 1; j >= i; --j) b[j] += d * b[j + 1];
    return b;
}

static double horner(const Coef &a, int deg, double u)
{
    double v = a[deg];
    for (int k = deg - 1; k >= 0; --k) v = v * u + a[k];
    return v;
}

static PPoly pp_box(double w)
{
    PPoly f;
    f.x = {-0.5 * w, 0.5 * w};
    Coef a{};
    a[0] = 1.0 / w;
    f.c = {a};
    f.deg = 0;
    return f;
}

static PPoly pp_convolve_box(const PPoly &f, double w)
{
    const int np = (int)f.c.size();
    const int D = f.deg + 1;
    // antiderivative, continuous, zero left of the support
    std::vector<Coef> Fc(np);
    double acc = 0.0;
    for (int i = 0; i < np; ++i) {
        Coef b{};
        b[0] = acc;
        for (int k = 0; k <= f.deg; ++k) b[k + 1] = f.c[i][k] / (k + 1);
        Fc[i] = b;
        acc = horner(b, D, f.x[i + 1] - f.x[i]);
    }
    const double total = acc;
    std::vector<double> z;
    z.reserve(2 * f.x.size());
    for (double v : f.x) {
        z.push_back(v - 0.5 * w);
        z.push_back(v + 0.5 * w);
    }
    std::sort(z.begin(), z.end());
    z.erase(std::unique(z.begin(), z.end()), z.end());
    // polynomial (in u = x - origin) of F(x + sh) on a piece around xm
    auto Fpoly = [&](double xm, double origin, double sh) {
        const double y = xm + sh;
        Coef r{};
        if (y <= f.x.front()) return r;
        if (y >= f.x.back()) {
            r[0] = total;
            return r;
        }
        int i = (int)(std::upper_bound(f.x.begin(), f.x.end(), y) - f.x.begin()) - 1;
        i = std::max(0, std::min(i, np - 1));
        return taylor_shift(Fc[i], D, origin + sh - f.x[i]);
    };
    PPoly g;
    g.deg = D;
    g.x = z;
    g.c.resize(z.size() - 1);
    for (size_t j = 0; j + 1 < z.size(); ++j) {
        const double xm = 0.5 * (z[j] + z[j + 1]);
        const Coef A = Fpoly(xm, z[j], 0.5 * w), B = Fpoly(xm, z[j], -0.5 * w);
        Coef r{};
        for (int k = 0; k <= D; ++k) r[k] = (A[k] - B[k]) / w;
        g.c[j] = r;
    }
    return g;
}

// Directions <= tol * max are treated as zero: a zero direction is the
// identity of convolution.
static PPoly pp_boxspline(std::vector<double> dirs, double scale)
{
    double mx = 0.0;
    for (double &d : dirs) {
        d = std::fabs(d);
        mx = std::max(mx, d);
    }
    std::vector<double> keep;
    for (double d : dirs)
        if (d > 1e-12 * mx) keep.push_back(d);
    std::sort(keep.begin(), keep.end());
    PPoly f = pp_box(keep[0]);
    for (size_t i = 1; i < keep.size(); ++i) f = pp_convolve_box(f, keep[i]);
    for (auto &c : f.c)
        for (double &v : c) v *= scale;
    return f;
}

static double pp_eval(const PPoly &f, double x)
{
    if (x <= f.x.front() || x >= f.x.back()) return 0.0;
    int i = (int)(std::upper_bound(f.x.begin(), f.x.end(), x) - f.x.begin()) - 1;
    i = std::max(0, std::min(i, (int)f.c.size() - 1));
    return horner(f.c[i], f.deg, x - f.x[i]);
}

// Sum of two piecewise polynomials: pieces on the union of the knots, each
// polynomial re-expanded about the merged piece's left knot.
static PPoly pp_add(const PPoly &f, const PPoly &g)
{
    PPoly h;
    h.deg = std::max(f.deg, g.deg);
    h.x = f.x;
    h.x.insert(h.x.end(), g.x.begin(), g.x.end());
    std::sort(h.x.begin(), h.x.end());
    h.x.erase(std::unique(h.x.begin(), h.x.end()), h.x.end());
    auto piece = [](const PPoly &q, double xm, double origin) {
        Coef r{};
        if (xm <= q.x.front() || xm >= q.x.back()) return r;
        int i = (int)(std::upper_bound(q.x.begin(), q.x.end(), xm) - q.x.begin()) - 1;
        i = std::max(0, std::min(i, (int)q.c.size() - 1));
        return taylor_shift(q.c[i], q.deg, origin - q.x[i]);
    };
    h.c.resize(h.x.size() - 1);
    for (size_t j = 0; j + 1 < h.x.size(); ++j) {
        const double xm = 0.5 * (h.x[j] + h.x[j + 1]);
        const Coef a = piece(f, xm, h.x[j]), b = piece(g, xm, h.x[j]);
        Coef r{};
        for (int k = 0; k <= h.deg; ++k) r[k] = a[k] + b[k];
        h.c[j] = r;
    }
    return h;
}

// ---------------------------------------------------------------------------
// Detector kernel (Sec. 2): boxes of widths w[i] with integrals a[i] (height
// times width), K(t) = sum_i (a[i] / w[i]) 1{|t| <= w[i]/2}.  No box: the
// point sample of the X-ray transform.  The paper's blur of width zeta is
// one box with a = 1.
// ---------------------------------------------------------------------------
struct Detector {
    std::vector<double> w, a;
    bool blurred() const { return !w.empty(); }
    double wmax() const
    {
        double m = 0.0;
        for (double v : w) m = std::max(m, v);
        return m;
    }
};

static Detector detector_of(double zeta)
{
    Detector D;
    if (zeta > 0.0) {
        D.w = {zeta};
        D.a = {1.0};
    }
    return D;
}

// ---------------------------------------------------------------------------
// Per-angle geometry.
// ---------------------------------------------------------------------------
struct AngleDirs {
    double c, s;      // cos, sin
    double a1, a2;    // l1|c|, l2|s| (exact zeros at axis-aligned angles)
    bool axis;
    int degree;       // B-spline degree of the interpolation (Sec. 5)
};

// Continuity rule of Sec. 5: the projected signal is C^0 in general and
// C^-1 at axis-aligned angles without blur; C^1 / C^0 with blur.  The
// interpolating B-spline degree is one above the continuity order.
static AngleDirs angle_dirs(double th, double l1, double l2, double zeta)  // zeta > 0: blurred
{
    AngleDirs d;
    d.c = std::cos(th);
    d.s = std::sin(th);
    d.axis = std::fabs(d.c) < 1e-12 || std::fabs(d.s) < 1e-12;
    d.a1 = std::fabs(d.c) < 1e-12 ? 0.0 : l1 * std::fabs(d.c);
    d.a2 = std::fabs(d.s) < 1e-12 ? 0.0 : l2 * std::fabs(d.s);
    if (zeta > 0.0) d.degree = d.axis ? 1 : 2;
    else d.degree = d.axis ? 0 : 1;
    return d;
}

static void sorted3(double a, double b, double c, double &L, double &M, double &S)
{
    double v[3] = {a, b, c};
    std::sort(v, v + 3);
    L = v[2];
    M = v[1];
    S = v[0];
}

// One term mult * (l1 l2)^2 * T_L * T_M * T_S of the Gram autocorrelation,
// {L, M, S} = sorted {l1|c|, l2|s|, zeta}.
template <typename T>
static GramAngle<T> gram_angle(const AngleDirs &d, double l1, double l2, double zeta, double mult = 1.0)
{
    GramAngle<T> g{};
    double L, M, S;
    sorted3(d.a1, d.a2, zeta, L, M, S);
    g.cx = l1 * d.c;
    g.sx = l2 * d.s;
    g.L = (T)L;
    g.M = (T)M;
    g.S = (T)S;
    g.iL2 = (T)(1.0 / (L * L));
    g.iM2 = M > 0 ? (T)(1.0 / (M * M)) : T(0);
    g.c6M = M > 0 ? (T)(1.0 / (6.0 * M * M)) : T(0);
    g.s12 = (T)(S * S / 12.0);
    g.c120S = S > 0 ? (T)(1.0 / (120.0 * S * S)) : T(0);
    g.scale = (T)(mult * l1 * l2 * l1 * l2);
    g.half = (T)(L + M + S);
    return g;
}

// Terms (hat half-width S, multiplier) of the Gram autocorrelation
// A = (l1 l2)^2 T_c * T_s * (K * K) (Sec. 4 with the kernel of Sec. 2).
// With box kernels B_w (unit integral, width w), K = sum_i a_i B_{w_i} and
// B_u * B_v = (s1^2 T_{s1} - s2^2 T_{s2}) / (u v), s1 = (u + v)/2,
// s2 = |u - v|/2 (the trapezoid as a difference of two hats), so every
// term is the six-direction closed form T_L * T_M * T_S.
static std::vector<std::array<double, 2>> gram_terms(const Detector &D)
{
    std::vector<std::array<double, 2>> t;
    if (!D.blurred()) return {{0.0, 1.0}};
    const size_t nb = D.w.size();
    for (size_t i = 0; i < nb; ++i) t.push_back({D.w[i], D.a[i] * D.a[i]});
    for (size_t i = 0; i < nb; ++i)
        for (size_t j = i + 1; j < nb; ++j) {
            const double u = D.w[i], v = D.w[j], f = 2.0 * D.a[i] * D.a[j] / (u * v);
            const double s1 = 0.5 * (u + v), s2 = 0.5 * std::fabs(u - v);
            t.push_back({s1, f * s1 * s1});
            if (s2 > 0.0) t.push_back({s2, -f * s2 * s2});
        }
    return t;
}

// Footprint term mult * l1 l2 M_[L, M, S] of one box (Sec. 4 eq. blurxray_of_f).
template <typename T>
static FwdAngle<T> fwd_angle(const AngleDirs &d, double l1, double l2, double zeta, double mult = 1.0)
{
    FwdAngle<T> f{};
    double L, M, S;
    sorted3(d.a1, d.a2, zeta, L, M, S);
    f.cx = l1 * d.c;
    f.sx = l2 * d.s;
    f.L = (T)L;
    f.M = (T)M;
    f.S = (T)S;
    f.iL = (T)(1.0 / L);
    f.iM = M > 0 ? (T)(1.0 / M) : T(0);
    f.i2MS = (M > 0 && S > 0) ? (T)(1.0 / (2.0 * M * S)) : T(0);
    f.scale_over_L = (T)(mult * l1 * l2 / L);
    f.half = (T)(0.5 * (L + M + S));
    f.rows = std::fabs(f.cx) >= std::fabs(f.sx) ? 1 : 0;
    return f;
}

// Back-projection kernel of one angle as sub-interval polynomials (see
// Whether G has the eight symmetries of the square (Sec. 4: G[k] sums
// A_theta(k1 l1 c + k2 l2 s), and A_theta depends on |c| and |s| alone, the
// same way on both): with square pixels, an angle set closed under
// theta -> theta + pi/2 and under theta -> -theta (mod pi, multiplicities
// included) makes G[k1][k2] = G[k2][-k1] = G[-k1][k2].  Uniform sets
// theta_i = i pi / n with n even qualify.  Angles are compared within 1e-14
// (a few units in the last place of pi): a tap at distance 2^11 then moves by
// less than 1e-10 of a bin.
static bool gram_symmetric(const double *theta, int n, double l1, double l2)
{
    if (l1 != l2 || n < 1) return false;
    const double tol = 1e-14;
    auto norm = [&](double t) {
        t = std::fmod(t, M_PI);
        if (t < 0.0) t += M_PI;
        if (t >= M_PI - tol) t = 0.0;  // pi is 0
        return t;
    };
    std::vector<double> a(n), r(n), m(n);
    for (int i = 0; i < n; ++i) {
        a[i] = norm(theta[i]);
        r[i] = norm(a[i] + 0.5 * M_PI);
        m[i] = norm(M_PI - a[i]);
    }
    std::sort(a.begin(), a.end());
    std::sort(r.begin(), r.end());
    std::sort(m.begin(), m.end());
    for (int i = 0; i < n; ++i)
        if (std::fabs(r[i] - a[i]) > tol || std::fabs(m[i] - a[i]) > tol) return false;
    return true;
}

// BPAngleHost).  coef is [nsub][J][D1] for this angle, J and D1 its own.
struct BPAngleTable {
    BPAngleHost h;
    std::vector<double> brk;   // nsub
    int J = 0, D1 = 0;
    std::vector<double> coef;  // nsub * J * D1
};

static BPAngleTable bp_angle(const AngleDirs &d, int N, double l1, double l2, double ly, int M,
                             const Detector &D)
{
    BPAngleTable t;
    // kappa = l1 l2 sum_i a_i M_{[l1|c|, l2|s|, w_i, ly x (d+1)] / ly}
    auto term = [&](double w, double a) {
        std::vector<double> dirs = {d.a1 / ly, d.a2 / ly, w / ly};
        for (int i = 0; i <= d.degree; ++i) dirs.push_back(1.0);
        return pp_boxspline(dirs, l1 * l2 * a);
    };
    PPoly k = D.blurred() ? term(D.w[0], D.a[0]) : term(0.0, 1.0);
    for (size_t i = 1; i < D.w.size(); ++i) k = pp_add(k, term(D.w[i], D.a[i]));
    // sub-interval breakpoints of t in [0,1): fractional parts of -knot
    std::vector<double> br = {0.0};
    for (double x : k.x) {
        double f = -x - std::floor(-x);
        if (f >= 1.0) f -= 1.0;
        br.push_back(f);
    }
    std::sort(br.begin(), br.end());
    std::vector<double> ub;
    for (double v : br)
        if (ub.empty() || v - ub.back() > 1e-12) ub.push_back(v);
    if (ub.size() > 1 && 1.0 - ub.back() <= 1e-12) ub.pop_back();
    t.brk = ub;
    const int nsub = (int)ub.size();
    const int jlo = (int)std::floor(k.x.front()) + 1;
    const int jhi = (int)std::ceil(k.x.back());
    t.J = jhi - jlo + 1;
    t.D1 = k.deg + 1;
    t.coef.assign((size_t)nsub * t.J * t.D1, 0.0);
    for (int s = 0; s < nsub; ++s) {
        const double lo = ub[s], hi = (s + 1 < nsub) ? ub[s + 1] : 1.0;
        for (int j = 0; j < t.J; ++j) {
            const double jj = jlo + j;
            const double xm = jj - 0.5 * (lo + hi);  // argument of kappa mid-interval
            if (xm <= k.x.front() || xm >= k.x.back()) continue;
            int i = (int)(std::upper_bound(k.x.begin(), k.x.end(), xm) - k.x.begin()) - 1;
            i = std::max(0, std::min(i, (int)k.c.size() - 1));
            // kappa(jj - lo - u) = P_i(delta - u), delta = jj - lo - x_i
            const Coef b = taylor_shift(k.c[i], k.deg, jj - lo - k.x[i]);
            for (int q = 0; q <= k.deg; ++q)
                t.coef[((size_t)s * t.J + j) * t.D1 + q] = (q & 1) ? -b[q] : b[q];
        }
    }
    t.h.nsub = nsub;
    t.h.jlo = jlo;
    t.h.degree = d.degree;
    t.h.dz1 = l1 * d.c / ly;
    t.h.dz2 = l2 * d.s / ly;
    t.h.z0 = -0.5 * (N - 1) * (t.h.dz1 + t.h.dz2) + 0.5 * (M - 1);
    return t;
}

template <typename T>
static int upload(void **dst, const std::vector<T> &v)
{
    if (v.empty()) return GCT_OK;
    hipError_t e = hipMalloc(dst, v.size() * sizeof(T));
    if (e != hipSuccess) return check_hip(e, "hipMalloc(plan tables)");
    e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return check_hip(e, "hipMemcpy(plan tables)");
}

template <typename T>
static std::vector<T> cast_vec(const std::vector<double> &v)
{
    return std::vector<T>(v.begin(), v.end());
}

static int build_plan(const gct_geometry *g, const Detector &det, gct_plan *p)
{
    const int n = g->n_angles;
    const double l1 = g->lambda_x[0], l2 = g->lambda_x[1], ly = g->lambda_y;
    std::vector<AngleDirs> ad(n);
    for (int a = 0; a < n; ++a) ad[a] = angle_dirs(g->theta[a], l1, l2, det.blurred() ? 1.0 : 0.0);
    // Gram terms per angle (entry a * nt + t) and footprint boxes per angle
    const auto terms = gram_terms(det);
    const int nt = (int)terms.size();
    const int nbf = det.blurred() ? (int)det.w.size() : 1;
    p->gram_n = n * nt;
    p->fwd_nb = nbf;

    std::vector<GramAngle<float>> gf((size_t)n * nt);
    std::vector<GramAngle<double>> gd((size_t)n * nt);
    std::vector<FwdAngle<float>> ff((size_t)n * nbf);
    std::vector<FwdAngle<double>> fd((size_t)n * nbf);
    std::vector<int32_t> deg(n);
    std::vector<BPAngleTable> bt(n);
    int smax = 1, J = 1, D1 = 1;
    double span = 0.0;
    for (int a = 0; a < n; ++a) {
        span = std::max(span, (ad[a].a1 + ad[a].a2) / ly);
        for (int t = 0; t < nt; ++t) {
            gf[(size_t)a * nt + t] = gram_angle<float>(ad[a], l1, l2, terms[t][0], terms[t][1]);
            gd[(size_t)a * nt + t] = gram_angle<double>(ad[a], l1, l2, terms[t][0], terms[t][1]);
        }
        for (int b = 0; b < nbf; ++b) {
            const double w = det.blurred() ? det.w[b] : 0.0, m = det.blurred() ? det.a[b] : 1.0;
            ff[(size_t)a * nbf + b] = fwd_angle<float>(ad[a], l1, l2, w, m);
            fd[(size_t)a * nbf + b] = fwd_angle<double>(ad[a], l1, l2, w, m);
        }
        deg[a] = ad[a].degree;
        bt[a] = bp_angle(ad[a], g->N, l1, l2, ly, g->M, det);
        smax = std::max(smax, bt[a].h.nsub);
        J = std::max(J, bt[a].J);
        D1 = std::max(D1, bt[a].D1);
    }
    p->bp.smax = smax;
    p->bp.J = J;
    p->bp.D1 = D1;
    p->bp.span_per_pixel = span;
    double win = 0.0;
    for (int a = 0; a < n; ++a)
        win = std::max(win, (BP_TX - 1) * std::fabs(bt[a].h.dz1) + (BP_TY - 1) * std::fabs(bt[a].h.dz2));
    p->bp.tile_win = win;
    std::vector<double> geo((size_t)n * 4, 0.0), brk((size_t)n * smax, 2.0);
    std::vector<int32_t> ints((size_t)n * 4, 0);
    std::vector<double> coef((size_t)n * smax * J * D1, 0.0);
    for (int a = 0; a < n; ++a) {
        const BPAngleTable &t = bt[a];
        geo[4 * a] = t.h.z0;
        geo[4 * a + 1] = t.h.dz1;
        geo[4 * a + 2] = t.h.dz2;
        ints[4 * a] = t.h.nsub;
        ints[4 * a + 1] = t.h.jlo;
        ints[4 * a + 2] = t.h.degree;
        // the device kernels evaluate each sub-interval's polynomial in the
        // offset t within the bin: sum_q c_q (t - b)^q re-expanded in powers
        // of t, d_k = sum_{q >= k} c_q C(q, k) (-b)^(q - k), in FP64
        for (int s = 0; s < t.h.nsub; ++s) {
            const double b = t.brk[s];
            brk[(size_t)a * smax + s] = b;
            for (int j = 0; j < t.J; ++j) {
                const double *c = &t.coef[((size_t)s * t.J + j) * t.D1];
                for (int k = 0; k < t.D1; ++k) {
                    double d = 0.0, binom = 1.0, pw = 1.0;  // C(q, k), (-b)^(q - k) at q = k
                    for (int q = k; q < t.D1; ++q) {
                        d += c[q] * binom * pw;
                        binom = binom * (q + 1) / (q + 1 - k);
                        pw *= -b;
                    }
                    coef[(((size_t)a * smax + s) * J + j) * D1 + k] = d;
                }
            }
        }
    }
    // rows of the back projection's per-angle interpolant tables: every bin
    // window of the tile grid (ragged tiles included: the grid's extent),
    // from two bins below the lowest projection to three above the highest;
    // the first row's bin per angle in ints[4 a + 3]
    {
        const double X1 = (double)(BP_TX * ((g->N + BP_TX - 1) / BP_TX) - 1);
        const double X2 = (double)(BP_TY * ((g->N + BP_TY - 1) / BP_TY) - 1);
        int MT = 1;
        for (int a = 0; a < n; ++a) {
            const double z0 = geo[4 * a], e1 = X1 * geo[4 * a + 1], e2 = X2 * geo[4 * a + 2];
            const double zmin = z0 + std::min(e1, 0.0) + std::min(e2, 0.0);
            const double zmax = z0 + std::max(e1, 0.0) + std::max(e2, 0.0);
            const int mA = (int)std::floor(zmin) - 2;
            ints[4 * a + 3] = mA;
            MT = std::max(MT, (int)std::floor(zmax) + 3 - mA);
        }
        p->bp.MT = MT;
    }
    // FFT twiddles e^{-2 pi i k / P}
    std::vector<double> tw((size_t)p->P);  // interleaved (re, im), P/2 entries
    for (int k = 0; k < p->P / 2; ++k) {
        const double ang = -2.0 * M_PI * (double)k / (double)p->P;
        tw[2 * k] = std::cos(ang);
        tw[2 * k + 1] = std::sin(ang);
    }
    // quadratic B-spline correction filter, Sec. 5: q[m] = sqrt2 (2 sqrt2 - 3)^|m|
    const int K = g->prefilter_K;
    std::vector<double> q(2 * K + 1);
    const double alpha = 2.0 * std::sqrt(2.0) - 3.0;
    for (int m = -K; m <= K; ++m) q[m + K] = std::sqrt(2.0) * std::pow(alpha, std::abs(m));

    // every table the plan keeps on the device, with its bytes counted
    auto up = [&](void **d, const auto &v) {
        p->dev_bytes += (int64_t)(v.size() * sizeof(v[0]));
        return upload(d, v);
    };
    int rc;
    if ((rc = up(&p->dev.gram_f32, gf))) return rc;
    if ((rc = up(&p->dev.gram_f64, gd))) return rc;
    {
        // Gram entries (angle, term) sorted by theta mod pi, for the Gram
        // build's angular windows (the terms of one angle stay together)
        const int ne = p->gram_n;
        std::vector<double> th(ne);
        std::vector<int32_t> ord(ne);
        double hmax = 0.0;
        for (int e = 0; e < ne; ++e) {
            double t = std::fmod(g->theta[e / nt], M_PI);
            if (t < 0.0) t += M_PI;
            if (t >= M_PI) t = 0.0;
            th[e] = t;
            ord[e] = e;
            hmax = std::max(hmax, (double)gd[e].half);
        }
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return th[x] < th[y]; });
        std::vector<double> ths(ne);
        for (int e = 0; e < ne; ++e) ths[e] = th[ord[e]];
        p->gram_hmax = hmax;
        p->gram_d4 = gram_symmetric(g->theta, n, l1, l2) ? 1 : 0;
        if ((rc = up(&p->dev.gram_ord, ord))) return rc;
        if ((rc = up(&p->dev.gram_th, ths))) return rc;
    }
    if ((rc = up(&p->dev.fwd_f32, ff))) return rc;
    if ((rc = up(&p->dev.fwd_f64, fd))) return rc;
    if ((rc = up(&p->dev.bp_geo, geo))) return rc;
    if ((rc = up(&p->dev.bp_int, ints))) return rc;
    if ((rc = up(&p->dev.bp_brk_f32, cast_vec<float>(brk)))) return rc;
    if ((rc = up(&p->dev.bp_brk_f64, brk))) return rc;
    if ((rc = up(&p->dev.bp_coef_f32, cast_vec<float>(coef)))) return rc;
    if ((rc = up(&p->dev.bp_coef_f64, coef))) return rc;
    if ((rc = up(&p->dev.tw_f32, cast_vec<float>(tw)))) return rc;
    if ((rc = up(&p->dev.tw_f64, tw))) return rc;
    if ((rc = up(&p->dev.q_f32, cast_vec<float>(q)))) return rc;
    if ((rc = up(&p->dev.q_f64, q))) return rc;
    if ((rc = up(&p->dev.deg, deg))) return rc;
    return GCT_OK;
}

static void free_tables(gct_plan *p)
{
    void **all[] = {&p->dev.gram_f32,    &p->dev.gram_f64,    &p->dev.fwd_f32,     &p->dev.fwd_f64,
                    &p->dev.bp_geo,      &p->dev.bp_int,      &p->dev.bp_brk_f32,  &p->dev.bp_brk_f64,
                    &p->dev.bp_coef_f32, &p->dev.bp_coef_f64, &p->dev.tw_f32,      &p->dev.tw_f64,
                    &p->dev.q_f32,       &p->dev.q_f64,       &p->dev.deg,         &p->dev.gram_ord,
                    &p->dev.gram_th};
    for (void **v : all) {
        if (*v) (void)hipFree(*v);
        *v = nullptr;
    }
}

static int validate(const gct_geometry *g, double wmax = -1.0)
{
    if (!g) return fail(GCT_EINVAL, "geometry is NULL");
    if (g->N < 1 || g->N > 2048) return fail(GCT_EINVAL, "N must be in [1, 2048]");
    if (g->n_angles < 1) return fail(GCT_EINVAL, "n_angles must be >= 1");
    if (!g->theta) return fail(GCT_EINVAL, "theta is NULL");
    if (g->M < 1) return fail(GCT_EINVAL, "M must be >= 1");
    if (!(g->lambda_x[0] > 0.0) || !(g->lambda_x[1] > 0.0) || !std::isfinite(g->lambda_x[0]) ||
        !std::isfinite(g->lambda_x[1]))
        return fail(GCT_EINVAL, "lambda_x must be finite and > 0");
    if (!(g->lambda_y > 0.0) || !std::isfinite(g->lambda_y))
        return fail(GCT_EINVAL, "lambda_y must be finite and > 0");
    if (!(g->zeta_blur >= 0.0) || !std::isfinite(g->zeta_blur))
        return fail(GCT_EINVAL, "zeta_blur must be finite and >= 0");
    if (g->prefilter_K < 0 || g->prefilter_K > 256)
        return fail(GCT_EINVAL, "prefilter_K must be in [0, 256]");
    for (int a = 0; a < g->n_angles; ++a)
        if (!std::isfinite(g->theta[a])) return fail(GCT_EINVAL, "theta contains a non-finite value");
    // back-projection table size: the kernel support in bins must stay modest
    const double w = (g->lambda_x[0] + g->lambda_x[1] + (wmax >= 0.0 ? wmax : g->zeta_blur)) / g->lambda_y + 3.0;
    if (w > 48.0) return fail(GCT_EINVAL, "lambda_y too small for the pixel size (kernel spans > 48 bins)");
    const double lratio = g->lambda_x[0] / g->lambda_x[1];
    if (lratio > 64.0 || lratio < 1.0 / 64.0) return fail(GCT_EINVAL, "pixel aspect ratio beyond 64");
    return GCT_OK;
}

}  // namespace gct

using namespace gct;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *gct_last_error(void) { return g_last_error.c_str(); }

static int create_plan(const gct_geometry *geom, const Detector &det, gct_plan **plan)
{
    int rc = GCT_OK;
    try {
        gct_plan *p = new gct_plan();
        p->N = geom->N;
        p->n = geom->n_angles;
        p->M = geom->M;
        p->K = geom->prefilter_K;
        p->lx1 = geom->lambda_x[0];
        p->lx2 = geom->lambda_x[1];
        p->ly = geom->lambda_y;
        p->zeta = geom->zeta_blur;
        int P, pc;
        choose_fft_size(p->N, P, pc);
        p->P = P;
        p->pc = pc;
        // elements per thread of the transform passes until gct_plan_autotune
        int er, ec;
        default_pass_elems(P, er, ec);
        p->fft_e[0] = p->fft_e[1] = p->cg_e[0] = p->cg_e[1] = er;
        p->fft_ec[0] = p->fft_ec[1] = p->cg_ec[0] = p->cg_ec[1] = ec;
        if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
        rc = build_plan(geom, det, p);
        if (rc) {
            free_tables(p);
            delete p;
            return rc;
        }
        bp_configure(p);
        *plan = p;
        return GCT_OK;
    } catch (const std::exception &e) {
        return fail(GCT_EINVAL, std::string("plan construction failed: ") + e.what());
    }
}

int gct_plan_create(const gct_geometry *geom, gct_plan **plan)
{
    if (!plan) return fail(GCT_EINVAL, "plan output pointer is NULL");
    *plan = nullptr;
    int rc = validate(geom);
    if (rc) return rc;
    return create_plan(geom, detector_of(geom->zeta_blur), plan);
}

int gct_plan_create_detector(const gct_geometry *geom, int32_t n_boxes, const double *box_width,
                             const double *box_height, gct_plan **plan)
{
    if (!plan) return fail(GCT_EINVAL, "plan output pointer is NULL");
    *plan = nullptr;
    if (!geom) return fail(GCT_EINVAL, "geometry is NULL");
    if (geom->zeta_blur != 0.0) return fail(GCT_EINVAL, "give the detector either as zeta_blur or as boxes");
    if (n_boxes < 1 || n_boxes > GCT_MAX_BOXES) return fail(GCT_EINVAL, "n_boxes must be in [1, 4]");
    if (!box_width || !box_height) return fail(GCT_EINVAL, "box arrays are NULL");
    Detector det;
    for (int i = 0; i < n_boxes; ++i) {
        if (!(box_width[i] > 0.0) || !std::isfinite(box_width[i]))
            return fail(GCT_EINVAL, "box widths must be finite and > 0");
        if (!std::isfinite(box_height[i]) || box_height[i] == 0.0)
            return fail(GCT_EINVAL, "box heights must be finite and non-zero");
        det.w.push_back(box_width[i]);
        det.a.push_back(box_width[i] * box_height[i]);
    }
    int rc = validate(geom, det.wmax());
    if (rc) return rc;
    return create_plan(geom, det, plan);
}

int gct_plan_destroy(gct_plan *plan)
{
    if (!plan) return GCT_OK;
    for (auto &g : plan->cg_graphs) (void)hipGraphExecDestroy(g.exec);
    plan->cg_graphs.clear();
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    if (plan->cg_pin) (void)hipHostFree(plan->cg_pin);
    if (plan->cg_ev) (void)hipEventDestroy(plan->cg_ev);
    free_tables(plan);
    delete plan;
    return GCT_OK;
}

int gct_plan_get_info(const gct_plan *p, gct_plan_info *info)
{
    if (!p || !info) return fail(GCT_EINVAL, "NULL argument");
    info->N = p->N;
    info->n_angles = p->n;
    info->M = p->M;
    info->prefilter_K = p->K;
    info->fft_size = p->P;
    info->gram_elems = (int64_t)(2 * p->N - 1) * (2 * p->N - 1);
    info->spectrum_elems = (int64_t)(p->P / 2 + 1) * p->P;
    info->image_elems = (int64_t)p->N * p->N;
    info->sino_elems = (int64_t)p->n * p->M;
    info->prefiltered_elems = (int64_t)p->n * (p->M + 2 * p->K);
    info->gram_symmetry = p->gram_d4 ? 8 : 2;
    return GCT_OK;
}

size_t gct_workspace_size(const gct_plan *p, int op, gct_dtype dt)
{
    if (!p) return 0;
    const size_t e = dt == GCT_F64 ? 8 : 4;
    switch (op) {
    case GCT_OP_GRAM_SPECTRUM: return spectrum_ws_bytes(p, e);
    case GCT_OP_GRAM_APPLY: return apply_ws_bytes(p, e);
    case GCT_OP_BACKPROJECT: return bp_workspace(p, e).total;
    case GCT_OP_CG: return cg_ws_bytes(p, e);
    default: return 0;
    }
}

#define CHECK_PLAN_DT(p, dt)                                                          \
    do {                                                                              \
        if (!(p)) return fail(GCT_EINVAL, "plan is NULL");                            \
        if ((dt) != GCT_F32 && (dt) != GCT_F64) return fail(GCT_EINVAL, "bad dtype"); \
    } while (0)

static bool misaligned(const void *ws) { return (reinterpret_cast<uintptr_t>(ws) & 255u) != 0; }

int gct_gram_build(const gct_plan *p, gct_dtype dt, void *G, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!G) return fail(GCT_EINVAL, "G is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32 ? launch_gram_build<float>(p, (float *)G, s)
                                 : launch_gram_build<double>(p, (double *)G, s);
    return check_hip(e, "gram_build launch");
}

int gct_gram_spectrum(const gct_plan *p, gct_dtype dt, const void *G, void *Ghat, void *ws,
                      void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!G || !Ghat || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (misaligned(ws)) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32
                       ? launch_gram_spectrum<float>(p, (const float *)G, (float *)Ghat, ws, s)
                       : launch_gram_spectrum<double>(p, (const double *)G, (double *)Ghat, ws, s);
    return check_hip(e, "gram_spectrum launch");
}

int gct_gram_apply(const gct_plan *p, gct_dtype dt, const void *Ghat, const void *c, void *y,
                   void *ws, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!Ghat || !c || !y || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (c == y) return fail(GCT_EINVAL, "y must not alias c");
    if (misaligned(ws)) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32 ? launch_gram_apply<float>(p, (const float *)Ghat, (const float *)c,
                                                            (float *)y, ws, s)
                                 : launch_gram_apply<double>(p, (const double *)Ghat,
                                                             (const double *)c, (double *)y, ws, s);
    return check_hip(e, "gram_apply launch");
}

int gct_prefilter(const gct_plan *p, gct_dtype dt, const void *g_s, void *out, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!g_s || !out) return fail(GCT_EINVAL, "NULL buffer");
    if (g_s == out) return fail(GCT_EINVAL, "output must not alias the sinogram");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32 ? launch_prefilter<float>(p, (const float *)g_s, (float *)out, s)
                                 : launch_prefilter<double>(p, (const double *)g_s, (double *)out, s);
    return check_hip(e, "prefilter launch");
}

int gct_backproject_boxspline(const gct_plan *p, gct_dtype dt, const void *g_s, void *b, void *ws,
                              void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!g_s || !b || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (misaligned(ws)) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    const BPWorkspace W = bp_workspace(p, dt == GCT_F32 ? 4 : 8);
    void *part = reinterpret_cast<char *>(ws) + W.part, *etab = reinterpret_cast<char *>(ws) + W.etab;
    if (dt == GCT_F32) {
        e = launch_prefilter<float>(p, (const float *)g_s, (float *)ws, s);
        if (e == hipSuccess)
            e = launch_backproject<float>(p, (const float *)ws, (float *)b, (float *)part, (float *)etab, s);
    } else {
        e = launch_prefilter<double>(p, (const double *)g_s, (double *)ws, s);
        if (e == hipSuccess)
            e = launch_backproject<double>(p, (const double *)ws, (double *)b, (double *)part, (double *)etab, s);
    }
    return check_hip(e, "backproject launch");
}

int gct_forward_project(const gct_plan *p, gct_dtype dt, const void *c, void *g_s, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!c || !g_s) return fail(GCT_EINVAL, "NULL buffer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dt == GCT_F32 ? launch_forward<float>(p, (const float *)c, (float *)g_s, s)
                                 : launch_forward<double>(p, (const double *)c, (double *)g_s, s);
    return check_hip(e, "forward_project launch");
}

int gct_cg_solve(const gct_plan *p, gct_dtype dt, const void *Ghat, const void *b, void *x,
                 int use_x0, double rtol, int32_t max_iter, int32_t check_every, double *hist,
                 gct_cg_result *res, void *ws, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!Ghat || !b || !x || !ws || !res) return fail(GCT_EINVAL, "NULL argument");
    if (b == x) return fail(GCT_EINVAL, "x must not alias b");
    if (max_iter < 0) return fail(GCT_EINVAL, "max_iter must be >= 0");
    if (!(rtol >= 0.0)) return fail(GCT_EINVAL, "rtol must be >= 0");
    if (misaligned(ws)) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    std::memset(res, 0, sizeof(*res));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = dt == GCT_F32 ? cg_solve<float>(p, (const float *)Ghat, (const float *)b, (float *)x,
                                             use_x0, rtol, max_iter, check_every, hist, res, ws, s)
                           : cg_solve<double>(p, (const double *)Ghat, (const double *)b,
                                              (double *)x, use_x0, rtol, max_iter, check_every,
                                              hist, res, ws, s);
    if (rc == GCT_ENOTCONV) set_error("cg_solve: max_iter reached before rtol");
    if (rc == GCT_EBREAKDOWN) set_error("cg_solve: breakdown (p.Ap <= 0 or non-finite value)");
    return rc;
}

int gct_sd_solve(const gct_plan *p, gct_dtype dt, const void *Ghat, const void *b, void *x,
                 int use_x0, double rtol, int32_t max_iter, int32_t check_every, double *hist,
                 gct_cg_result *res, void *ws, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!Ghat || !b || !x || !ws || !res) return fail(GCT_EINVAL, "NULL argument");
    if (b == x) return fail(GCT_EINVAL, "x must not alias b");
    if (max_iter < 0) return fail(GCT_EINVAL, "max_iter must be >= 0");
    if (!(rtol >= 0.0)) return fail(GCT_EINVAL, "rtol must be >= 0");
    if (misaligned(ws)) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    std::memset(res, 0, sizeof(*res));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = dt == GCT_F32 ? cg_solve<float>(p, (const float *)Ghat, (const float *)b, (float *)x,
                                             use_x0, rtol, max_iter, check_every, hist, res, ws, s, 1)
                           : cg_solve<double>(p, (const double *)Ghat, (const double *)b,
                                              (double *)x, use_x0, rtol, max_iter, check_every,
                                              hist, res, ws, s, 1);
    if (rc == GCT_ENOTCONV) set_error("sd_solve: max_iter reached before rtol");
    if (rc == GCT_EBREAKDOWN) set_error("sd_solve: breakdown (r.Ar <= 0 or non-finite value)");
    return rc;
}

int gct_plan_set_pass_elems(gct_plan *p, gct_dtype dt, int32_t Er, int32_t Ec)
{
    CHECK_PLAN_DT(p, dt);
    int dr, dc;
    default_pass_elems(p->P, dr, dc);
    if (Er == 0) Er = dr;
    if (Ec == 0) Ec = dc;
    if (!apply_e_ok(p->pc, Er) || !apply_e_ok(p->pc, Ec))
        return fail(GCT_EINVAL, "elements per thread not available for this transform size");
    const int t = dt == GCT_F32 ? 0 : 1;
    if (p->fft_e[t] != Er || p->fft_ec[t] != Ec || p->cg_e[t] != Er || p->cg_ec[t] != Ec) {
        p->fft_e[t] = p->cg_e[t] = Er;
        p->fft_ec[t] = p->cg_ec[t] = Ec;
        for (auto &g : p->cg_graphs) (void)hipGraphExecDestroy(g.exec);
        p->cg_graphs.clear();
    }
    return GCT_OK;
}

int gct_plan_set_fft_elems(gct_plan *p, gct_dtype dt, int32_t E)
{
    return gct_plan_set_pass_elems(p, dt, E, E);
}

int gct_plan_get_pass_elems(const gct_plan *p, gct_dtype dt, int32_t *out)
{
    CHECK_PLAN_DT(p, dt);
    if (!out) return fail(GCT_EINVAL, "NULL output");
    const int t = dt == GCT_F32 ? 0 : 1;
    out[0] = p->fft_e[t];
    out[1] = p->fft_ec[t];
    out[2] = p->cg_e[t];
    out[3] = p->cg_ec[t];
    return GCT_OK;
}

int gct_plan_device_bytes(const gct_plan *p, int64_t *bytes)
{
    if (!p || !bytes) return fail(GCT_EINVAL, "NULL argument");
    *bytes = p->dev_bytes;
    return GCT_OK;
}

int gct_plan_get_bp_shape(const gct_plan *p, gct_dtype dt, int32_t *out)
{
    CHECK_PLAN_DT(p, dt);
    if (!out) return fail(GCT_EINVAL, "NULL output");
    const int t = dt == GCT_F32 ? 0 : 1;
    const size_t e = dt == GCT_F32 ? 4 : 8;
    out[0] = p->bp_ch[t];
    out[1] = p->bp_ch[t] > 0 ? p->bp_groups[t] : 1;
    out[2] = p->bp_ch[t] > 0 ? 0 : bp_fallback_tile(p, e);
    out[3] = p->bp_ch[t] > 0 ? bp_breakpoint_regs(p, e) : 0;
    return GCT_OK;
}

int gct_plan_autotune(gct_plan *p, gct_dtype dt, const void *Ghat, void *ws, int32_t reps,
                      int32_t *chosen, void *stream)
{
    CHECK_PLAN_DT(p, dt);
    if (!Ghat || !ws) return fail(GCT_EINVAL, "NULL buffer");
    if (misaligned(ws)) return fail(GCT_EINVAL, "workspace must be 256-byte aligned");
    if (reps < 1) reps = 3;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return dt == GCT_F32 ? plan_autotune<float>(p, (const float *)Ghat, ws, reps, chosen, s)
                         : plan_autotune<double>(p, (const double *)Ghat, ws, reps, chosen, s);
}

// ---------------------------------------------------------------------------
// Host-only helpers (include/gramct_host.h)
// ---------------------------------------------------------------------------
int gct_host_boxspline_eval(const double *dirs, int ndirs, double scale, const double *x, int npts,
                            double *out)
{
    if (!dirs || ndirs < 1 || !x || !out || npts < 0) return fail(GCT_EINVAL, "bad argument");
    std::vector<double> d(dirs, dirs + ndirs);
    double mx = 0.0;
    for (double v : d) mx = std::max(mx, std::fabs(v));
    if (!(mx > 0.0)) return fail(GCT_EINVAL, "all directions are zero");
    if (ndirs > PP_MAXC - 2) return fail(GCT_EINVAL, "too many directions");
    try {
        const PPoly f = pp_boxspline(d, scale);
        for (int i = 0; i < npts; ++i) out[i] = pp_eval(f, x[i]);
    } catch (const std::exception &e) {
        return fail(GCT_EINVAL, e.what());
    }
    return GCT_OK;
}

int gct_host_bp_weights(const gct_geometry *g, int angle, double t, double *w, int *jlo, int *nw)
{
    int rc = validate(g);
    if (rc) return rc;
    if (angle < 0 || angle >= g->n_angles || !w || !jlo || !nw || !(t >= 0.0 && t < 1.0))
        return fail(GCT_EINVAL, "bad argument");
    const AngleDirs d = angle_dirs(g->theta[angle], g->lambda_x[0], g->lambda_x[1], g->zeta_blur);
    const BPAngleTable tb = bp_angle(d, g->N, g->lambda_x[0], g->lambda_x[1], g->lambda_y, g->M,
                                     detector_of(g->zeta_blur));
    int s = 0;
    for (int i = 1; i < tb.h.nsub; ++i)
        if (t >= tb.brk[i]) s = i;
    const double u = t - tb.brk[s];
    for (int j = 0; j < tb.J; ++j) {
        double v = 0.0;
        for (int q = tb.D1 - 1; q >= 0; --q) v = v * u + tb.coef[((size_t)s * tb.J + j) * tb.D1 + q];
        w[j] = v;
    }
    *jlo = tb.h.jlo;
    *nw = tb.J;
    return GCT_OK;
}

int gct_host_degree(double theta, double zeta_blur)
{
    return angle_dirs(theta, 1.0, 1.0, zeta_blur).degree;
}

}  // extern "C"
