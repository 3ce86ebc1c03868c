// Learned warm start for CG: a small U-Net mapping the normalised back
// projection H^T g to an initial iterate, trained and run entirely by the
// kernels in this file.
//
// Architecture (levels L, base channels C0; C_l = C0 2^l): per level two
// 3x3 convolutions with ReLU, 2x2 max pooling between encoder levels, 2x2
// stride-2 transposed convolution up, skip concatenation, final 1x1
// convolution to one channel.  Activations and weights are BF16 (NHWC),
// accumulation FP32 on the matrix cores (v_mfma_f32_16x16x16_bf16), master
// weights and Adam moments FP32.
//
// Every GEMM-shaped step is one implicit-GEMM kernel (k_conv): rows = output
// pixels, columns = output channels, K = taps x input channels, operands
// gathered straight from the NHWC tensors (zero padding by predication).
// The data gradient of a convolution is the same kernel with flipped,
// transposed weights; the weight gradient is a K-split GEMM over pixels
// (k_wgrad) reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gramct_unet.h"
#include "gct_internal.h"

namespace gct {

typedef uint16_t bf16_t;
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__host__ __device__ inline float bf2f(bf16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// round to nearest even
__host__ __device__ inline bf16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

__device__ inline short4_t load_bf4(const bf16_t *p)
{
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    short4_t r;
    r[0] = (short)(v.x & 0xffff);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffff);
    r[3] = (short)(v.y >> 16);
    return r;
}

// ---------------------------------------------------------------------------
// Implicit-GEMM convolution.  Rows m = (b, oh, ow) over the output grid
// Hout x Wout; for tap t the input pixel is (oh*stride + t/tw + org,
// ow*stride + t%tw + org); weights w[t][n][Cin] (Cin contiguous).
// Epilogue modes: 0 = BF16 NHWC (+bias, ReLU) at channel offset out_co of
// pixels with out_cs channels; 1 = FP32 single channel n = 0; 2 = stride-2
// transposed-convolution scatter: n = (2a + b) cout + co goes to output
// pixel (2 oh + a, 2 ow + b) of a 2Hout x 2Wout grid, channel out_co + co.
// Block: 4 waves x (16 rows x 64 columns); K in steps of 16 channels.
// ---------------------------------------------------------------------------
struct ConvArgs {
    const bf16_t *in;
    int in_cs, in_co;
    int B, Hin, Win, Cin;
    int ntaps, tw, org, stride;
    const bf16_t *w;
    int Nw;
    int Hout, Wout;
    const float *bias;
    int relu, mode;
    bf16_t *out;
    int out_cs, out_co;
    float *out32;
    float oscale;
    int cout;
    // direct kernel only: FP32 single-channel input (first layer) and the
    // final 1x1 layer fused into the epilogue (mode 3)
    const float *in32;
    float in_scale;
    const bf16_t *fw;
    const float *fb;
};

// Bias of GEMM column n (0 without bias).
__device__ inline float conv_bias(const ConvArgs &a, int n)
{
    if (!a.bias) return 0.f;
    return a.bias[a.mode == 2 ? n % a.cout : (a.mode == 1 ? 0 : n)];
}

// Epilogue of GEMM element (m, n) with accumulated value v and the bias bn
// of column n (modes above).
__device__ inline void conv_store(const ConvArgs &a, int m, int n, float v, float bn)
{
    v += bn;
    if (a.mode == 0) {
        if (a.relu) v = fmaxf(v, 0.f);
        a.out[(size_t)m * a.out_cs + a.out_co + n] = f2bf(v);
    } else if (a.mode == 1) {
        if (n == 0) a.out32[m] = a.oscale * v;
    } else {
        const int HWo = a.Hout * a.Wout;
        const int bb = m / HWo, rr = m - bb * HWo, yh = rr / a.Wout, yw = rr - yh * a.Wout;
        const int ab = n / a.cout, co = n - ab * a.cout;
        const int oy = 2 * yh + (ab >> 1), ox = 2 * yw + (ab & 1);
        if (a.relu) v = fmaxf(v, 0.f);
        const size_t pix = ((size_t)bb * (2 * a.Hout) + oy) * (2 * a.Wout) + ox;
        a.out[pix * a.out_cs + a.out_co + co] = f2bf(v);
    }
}

__global__ void __launch_bounds__(256) k_conv(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HWo = a.Hout * a.Wout;
    const int M = a.B * HWo;
    const int m0 = blockIdx.x * 64 + wave * 16;
    const int n0 = blockIdx.y * 64;
    const int mi = m0 + (lane & 15);
    const bool mvalid = mi < M;
    int b = 0, oh = 0, ow = 0;
    if (mvalid) {
        b = mi / HWo;
        const int r = mi - b * HWo;
        oh = r / a.Wout;
        ow = r - oh * a.Wout;
    }
    const int kq = (lane >> 4) * 4;
    float4_t acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = float4_t{0.f, 0.f, 0.f, 0.f};
    const short4_t zero = {0, 0, 0, 0};
    float bq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = n0 + 16 * q + (lane & 15);
        bq[q] = n < a.Nw ? conv_bias(a, n) : 0.f;
    }
    for (int t = 0; t < a.ntaps; ++t) {
        const int ih = oh * a.stride + t / a.tw + a.org;
        const int iw = ow * a.stride + t % a.tw + a.org;
        const bool ok = mvalid && ih >= 0 && ih < a.Hin && iw >= 0 && iw < a.Win;
        const bf16_t *ip = a.in + ((size_t)(b * a.Hin + (ok ? ih : 0)) * a.Win + (ok ? iw : 0)) * a.in_cs +
                           a.in_co + kq;
        const bf16_t *wp = a.w + ((size_t)t * a.Nw + n0 + (lane & 15)) * a.Cin + kq;
        for (int c0 = 0; c0 < a.Cin; c0 += 16) {
            const short4_t av = ok ? load_bf4(ip + c0) : zero;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = n0 + 16 * q + (lane & 15);
                const short4_t bv = n < a.Nw ? load_bf4(wp + (size_t)16 * q * a.Cin + c0) : zero;
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
    // D[i][n]: lane holds n = lane % 16, i = 4 (lane / 16) + j
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = n0 + 16 * q + (lane & 15);
        if (n >= a.Nw) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + (lane >> 4) * 4 + j;
            if (m < M) conv_store(a, m, n, acc[q][j], bq[q]);
        }
    }
}


// ---------------------------------------------------------------------------
// LDS-tiled implicit GEMM for the same convolutions (every mode but the
// one-column final layer).  Block tile BM x BN, K in steps of 32
// (v_mfma_f32_16x16x32_bf16), 4 waves as 2 x 2, each wave (BM/2) x (BN/2).
// K index k = t Cin + c; Cin is a multiple of 16, so each group of 8
// consecutive k (one 16-byte load) lies in one tap; the last step of a
// ragged K is zero-filled.  Operands are staged global -> registers -> LDS
// in chunks of 4 steps (one barrier pair per chunk, the next chunk's loads
// in flight during the MFMAs).  With gridDim.z > 1 the K steps are split
// over z and FP32 partials part[z][m][n] are reduced by k_conv_splitk in a
// fixed order.  (A reduction by the last block of each tile would need a
// device-scope release per block, i.e. an L2 write-back, which costs more
// than the extra launch.)
// Input gathers (IN): 0 = BF16 NHWC; 1 = the 2x2 max pool of a BF16 NHWC
// tensor of twice the grid (a.in un-pooled, a.Hin x a.Win the pooled grid:
// pooling fused into its consumer); 2 = FP32 single-channel image a.in32
// times in_scale, BF16-rounded into channel 0 of Cin = 16 (input
// preparation fused into the first layer).  Mode 3 = mode 0 plus the final
// 1x1 convolution of the stored BF16 activation, out32[m] = oscale (sum_n
// act[m][n] fw[n] + fb[0]); it needs every column in this block (Nw <= BN)
// and no K split.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ inline uint4 bf8_max(uint4 p, uint4 q)
{
    uint4 r;
    const uint32_t *x = &p.x, *y = &q.x;
    uint32_t *o = &r.x;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const float lo = fmaxf(__uint_as_float(x[w] << 16), __uint_as_float(y[w] << 16));
        const float hi = fmaxf(__uint_as_float(x[w] & 0xffff0000u), __uint_as_float(y[w] & 0xffff0000u));
        o[w] = (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
    }
    return r;
}

template <int BM, int BN, int IN>
__global__ void __launch_bounds__(256) k_conv2(ConvArgs a, int ksplit_steps, float *part)
{
    constexpr int NA = IN == 1 ? 4 : 1;  // loads per A chunk (the pooled 2x2 window)
    constexpr int LDK = 40;  // 32 + 8 padding bf16: 80-byte rows, conflict-free 16-byte reads
    constexpr int KC = 4;    // K steps staged per barrier (their loads are in flight together)
    constexpr int AP = BM * 4 / 256;            // A chunks per thread and step
    constexpr int BP = (BN * 4 + 255) / 256;    // B chunks per thread and step
    constexpr int TM = BM / 32, TN = BN / 32;   // 16x16 tiles per wave
    __shared__ __attribute__((aligned(16))) bf16_t sA[KC][BM * LDK];
    __shared__ __attribute__((aligned(16))) bf16_t sB[KC][BN * LDK];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int HWo = a.Hout * a.Wout, M = a.B * HWo;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int K = a.ntaps * a.Cin, nks = (K + 31) / 32;
    const int kbeg = blockIdx.z * ksplit_steps, kend = min(nks, kbeg + ksplit_steps);
    const int g = tid & 3;
    const int Ws = IN == 1 ? 2 * a.Win : a.Win;  // width of the gathered grid

    // per-thread rows (A) and columns (B)
    int rb[AP], rh[AP], rw[AP];
    bool rok[AP];
#pragma unroll
    for (int i = 0; i < AP; ++i) {
        const int m = m0 + (tid >> 2) + 64 * i;
        rok[i] = m < M;
        const int mm = rok[i] ? m : 0;
        const int b = mm / HWo, r = mm - b * HWo, oh = r / a.Wout, ow = r - oh * a.Wout;
        rb[i] = b * (IN == 1 ? 2 * a.Hin : a.Hin);
        rh[i] = oh * a.stride + a.org;
        rw[i] = ow * a.stride + a.org;
    }
    bool cok[BP];
    int cn[BP];
#pragma unroll
    for (int i = 0; i < BP; ++i) {
        const int q = tid + 256 * i;
        cn[i] = n0 + (q >> 2);
        cok[i] = q < BN * 4 && cn[i] < a.Nw;
    }
    // k state of this thread's 8-group in the next step to load: k = ks 32 + 8 g
    int kn = kbeg;
    int t, c, dy, dx;
    {
        const int k = kbeg * 32 + 8 * g;
        t = k / a.Cin;
        c = k - t * a.Cin;
        dy = t / a.tw;
        dx = t - dy * a.tw;
    }
    uint4 ra[KC][AP][NA], rbv[KC][BP];
    // issue the loads of steps kn .. kn + KC - 1 (zero past kend or K)
    auto gload = [&]() {
#pragma unroll
        for (int s = 0; s < KC; ++s) {
            const bool kok = t < a.ntaps && kn + s < kend;
#pragma unroll
            for (int i = 0; i < AP; ++i) {
                const int ih = rh[i] + dy, iw = rw[i] + dx;
                const bool ok = kok && rok[i] && ih >= 0 && ih < a.Hin && iw >= 0 && iw < a.Win;
                if (IN == 0) {
                    ra[s][i][0] = ok ? *reinterpret_cast<const uint4 *>(
                                           a.in + ((size_t)(rb[i] + ih) * a.Win + iw) * a.in_cs + a.in_co + c)
                                     : make_uint4(0, 0, 0, 0);
                } else if (IN == 1) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        ra[s][i][q] = ok ? *reinterpret_cast<const uint4 *>(
                                               a.in + ((size_t)(rb[i] + 2 * ih + (q >> 1)) * Ws + 2 * iw + (q & 1)) *
                                                          a.in_cs +
                                               a.in_co + c)
                                         : make_uint4(0, 0, 0, 0);
                } else {
                    // the pixel's FP32 value, converted when staged
                    ra[s][i][0].x = (ok && c == 0) ? __float_as_uint(a.in32[(size_t)(rb[i] + ih) * a.Win + iw]) : 0u;
                }
            }
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const bool ok = kok && cok[i];
                rbv[s][i] = ok ? *reinterpret_cast<const uint4 *>(a.w + ((size_t)t * a.Nw + cn[i]) * a.Cin + c)
                               : make_uint4(0, 0, 0, 0);
            }
            c += 32;
            while (c >= a.Cin) {
                c -= a.Cin;
                ++t;
                if (++dx == a.tw) {
                    dx = 0;
                    ++dy;
                }
            }
        }
        kn += KC;
    };

    float4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

    // epilogue columns of this lane: bias loaded now, while the K loop runs
    // (a load per stored element would wait out one memory latency each)
    float bcol[TN];
    int ccol[TN], acol[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int n = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
        acol[j] = a.mode == 2 ? n / a.cout : 0;
        ccol[j] = n - acol[j] * a.cout * (a.mode == 2);
        bcol[j] = (gridDim.z == 1 && a.bias && n < a.Nw) ? a.bias[ccol[j]] : 0.f;
    }

    if (kbeg < kend) gload();
    for (int ks0 = kbeg; ks0 < kend; ks0 += KC) {
        if (ks0 != kbeg) __syncthreads();  // the previous chunk's reads are done
#pragma unroll
        for (int s = 0; s < KC; ++s) {
#pragma unroll
            for (int i = 0; i < AP; ++i) {
                uint4 v = ra[s][i][0];
                if (IN == 1) v = bf8_max(bf8_max(ra[s][i][0], ra[s][i][1]), bf8_max(ra[s][i][2], ra[s][i][3]));
                if (IN == 2) v = make_uint4(f2bf(__uint_as_float(ra[s][i][0].x) * a.in_scale), 0u, 0u, 0u);
                *reinterpret_cast<uint4 *>(&sA[s][((tid >> 2) + 64 * i) * LDK + 8 * g]) = v;
            }
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const int q = tid + 256 * i;
                if (q < BN * 4) *reinterpret_cast<uint4 *>(&sB[s][(q >> 2) * LDK + 8 * g]) = rbv[s][i];
            }
        }
        __syncthreads();
        if (ks0 + KC < kend) gload();
        const int ns = min(KC, kend - ks0);
#pragma unroll
        for (int s = 0; s < KC; ++s) {
            if (s >= ns) break;
            bf16x8_t af[TM], bfr[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const bf16x8_t *>(
                    &sA[s][(wm * (BM / 2) + i * 16 + (lane & 15)) * LDK + (lane >> 4) * 8]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8_t *>(
                    &sB[s][(wn * (BN / 2) + j * 16 + (lane & 15)) * LDK + (lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
    }
    // D layout: row 4 (lane / 16) + r, column lane % 16 of each 16x16 tile
    if (gridDim.z == 1) {
        if (a.mode == 0) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int n = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
                    if (n >= a.Nw) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = m0 + wm * (BM / 2) + i * 16 + (lane >> 4) * 4 + r;
                        float v = acc[i][j][r] + bcol[j];
                        if (a.relu) v = fmaxf(v, 0.f);
                        if (m < M) a.out[(size_t)m * a.out_cs + a.out_co + n] = f2bf(v);
                    }
                }
        } else if (a.mode == 3) {
            // the block holds every column: row sums of act x fw over this
            // wave's columns (16 lanes per row), then over the two column
            // halves through LDS
            __shared__ float fsum[2][BM];
            float fwc[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = wn * (BN / 2) + j * 16 + (lane & 15);
                fwc[j] = n < a.Nw ? bf2f(a.fw[n]) : 0.f;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ml = wm * (BM / 2) + i * 16 + (lane >> 4) * 4 + r, m = m0 + ml;
                    float f = 0.f;
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const int n = wn * (BN / 2) + j * 16 + (lane & 15);
                        float v = acc[i][j][r] + bcol[j];
                        if (a.relu) v = fmaxf(v, 0.f);
                        const bf16_t h = f2bf(v);
                        if (m < M && n < a.Nw) a.out[(size_t)m * a.out_cs + a.out_co + n] = h;
                        f += bf2f(h) * fwc[j];
                    }
#pragma unroll
                    for (int o = 1; o < 16; o <<= 1) f += __shfl_xor(f, o, 16);
                    if ((lane & 15) == 0) fsum[wn][ml] = f;
                }
            __syncthreads();
            if (tid < BM && m0 + tid < M) a.out32[m0 + tid] = a.oscale * (fsum[0][tid] + fsum[1][tid] + a.fb[0]);
        } else {
            // transposed-convolution scatter: n = (2a + b) cout + co to output
            // pixel (2 oh + a, 2 ow + b)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m0 + wm * (BM / 2) + i * 16 + (lane >> 4) * 4 + r;
                    if (m >= M) continue;
                    const int bb = m / HWo, rr = m - bb * HWo, yh = rr / a.Wout, yw = rr - yh * a.Wout;
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const int n = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
                        if (n >= a.Nw) continue;
                        float v = acc[i][j][r] + bcol[j];
                        if (a.relu) v = fmaxf(v, 0.f);
                        const int oy = 2 * yh + (acol[j] >> 1), ox = 2 * yw + (acol[j] & 1);
                        const size_t pix = ((size_t)bb * (2 * a.Hout) + oy) * (2 * a.Wout) + ox;
                        a.out[pix * a.out_cs + a.out_co + ccol[j]] = f2bf(v);
                    }
                }
        }
        return;
    }
    // split K: partial tile to part[z][m][n], reduced by k_conv_splitk
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int n = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
            if (n >= a.Nw) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * (BM / 2) + i * 16 + (lane >> 4) * 4 + r;
                if (m < M) part[((size_t)blockIdx.z * M + m) * a.Nw + n] = acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------------------
// 3x3 convolution (stride 1, zero padding 1) from an LDS halo tile.  The
// gathered implicit GEMM above reads every input pixel once per tap (nine
// times) from L2; here a group of 4 waves stages its output tile's input
// window with the one-pixel halo, (TY + 2) x 18 pixels x 32 channels, once
// per chunk of 32 input channels, plus the chunk's weights for all nine
// taps and BN columns, and the nine taps read the window from LDS at
// shifted offsets.  Output tile: TY x 16 pixels of one image x BN channels;
// the 4 waves of a group as 2 x 2 (each (8 TY) rows x BN/2 columns; a
// 16-row MFMA tile is one image row of the tile).  The next chunk's loads
// are in flight (registers) during the current chunk's MFMAs.  A block
// holds KG such groups, which take every KG-th chunk and add their partial
// tiles into group 0's through LDS in group order (a fixed order), so short
// grids of long-K layers keep several waves per SIMD without a second
// launch.  Needs Cin to be a multiple of 32.  Input gathers IN 0 and 1 and
// epilogue modes 0 and 3 as in k_conv2.
// ---------------------------------------------------------------------------
template <int TY, int BN, int IN, int KG>
__global__ void __launch_bounds__(256 * KG) k_conv33(ConvArgs a)
{
    constexpr int LDK = 40;                        // 32 channels + 8 padding (80-byte rows)
    constexpr int HW_ = 18, HP = (TY + 2) * HW_;   // halo window width and pixels
    constexpr int MT = TY * 16;                    // output pixels per block
    constexpr int TM = MT / 32, TN = BN / 32;      // 16x16 tiles per wave
    constexpr int NA = IN == 1 ? 4 : 1;
    constexpr int PI = (HP * 4 + 255) / 256;       // input pieces (16 B) per thread
    constexpr int PW = (9 * BN * 4 + 255) / 256;   // weight pieces per thread
    constexpr int SG = (HP + 9 * BN) * LDK;        // bf16 of LDS per group
    static_assert((KG - 1) * 256 * TM * TN * 4 * 4 <= KG * SG * 2, "reduction area");
    __shared__ __attribute__((aligned(16))) bf16_t smem[KG * SG];

    const int tid = threadIdx.x & 255, grp = threadIdx.x >> 8;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int l16 = lane & 15, kg = lane >> 4;
    bf16_t *sIn = smem + grp * SG, *sW = sIn + HP * LDK;
    const int H = a.Hout, W = a.Wout;
    const int tx_n = (W + 15) / 16, ty_n = (H + TY - 1) / TY;
    const int bx = blockIdx.x % tx_n, by = (blockIdx.x / tx_n) % ty_n, b = blockIdx.x / (tx_n * ty_n);
    const int x0 = bx * 16, y0 = by * TY, n0 = blockIdx.y * BN;
    const int nch = a.Cin / 32;
    const int Hs = IN == 1 ? 2 * H : H, Ws = IN == 1 ? 2 * W : W;

    uint4 ri[PI][NA], rw[PW];
    auto gload = [&](int ch) {
        const int c0 = ch * 32;
#pragma unroll
        for (int q = 0; q < PI; ++q) {
            const int pc = tid + 256 * q, hp = pc >> 2, cg = pc & 3;
            const int yy = y0 - 1 + hp / HW_, xx = x0 - 1 + hp % HW_;
            const bool ok = pc < HP * 4 && yy >= 0 && yy < H && xx >= 0 && xx < W;
            if (IN == 0) {
                ri[q][0] = ok ? *reinterpret_cast<const uint4 *>(a.in + ((size_t)(b * Hs + yy) * Ws + xx) * a.in_cs +
                                                                 a.in_co + c0 + 8 * cg)
                              : make_uint4(0, 0, 0, 0);
            } else {
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    ri[q][w] = ok ? *reinterpret_cast<const uint4 *>(
                                        a.in + ((size_t)(b * Hs + 2 * yy + (w >> 1)) * Ws + 2 * xx + (w & 1)) * a.in_cs +
                                        a.in_co + c0 + 8 * cg)
                                  : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            const int pc = tid + 256 * q, row = pc >> 2, cg = pc & 3;  // row = tap BN + n
            const int tap = row / BN, n = n0 + row % BN;
            const bool ok = pc < 9 * BN * 4 && n < a.Nw;
            rw[q] = ok ? *reinterpret_cast<const uint4 *>(a.w + ((size_t)tap * a.Nw + n) * a.Cin + c0 + 8 * cg)
                       : make_uint4(0, 0, 0, 0);
        }
    };

    float4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    // epilogue columns of this lane
    float bcol[TN], fwc[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int n = n0 + wn * (BN / 2) + j * 16 + l16;
        bcol[j] = (a.bias && n < a.Nw) ? a.bias[n] : 0.f;
        fwc[j] = (a.mode == 3 && n < a.Nw) ? bf2f(a.fw[n]) : 0.f;
    }

    // group grp takes chunks grp, grp + KG, ...; every group runs the same
    // number of rounds (and barriers)
    const int rounds = (nch + KG - 1) / KG;
    if (grp < nch) gload(grp);
    for (int it = 0; it < rounds; ++it) {
        const int ch = it * KG + grp;
        const bool live = ch < nch;
        if (it != 0) __syncthreads();  // the previous round's LDS reads are done
        if (live) {
#pragma unroll
            for (int q = 0; q < PI; ++q) {
                const int pc = tid + 256 * q;
                uint4 v = ri[q][0];
                if (IN == 1) v = bf8_max(bf8_max(ri[q][0], ri[q][1]), bf8_max(ri[q][2], ri[q][3]));
                if (pc < HP * 4) *reinterpret_cast<uint4 *>(&sIn[(pc >> 2) * LDK + 8 * (pc & 3)]) = v;
            }
#pragma unroll
            for (int q = 0; q < PW; ++q) {
                const int pc = tid + 256 * q;
                if (pc < 9 * BN * 4) *reinterpret_cast<uint4 *>(&sW[(pc >> 2) * LDK + 8 * (pc & 3)]) = rw[q];
            }
        }
        __syncthreads();
        if (ch + KG < nch) gload(ch + KG);
        if (live) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;
                bf16x8_t af[TM], bfr[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int py = (wm * (MT / 2) + i * 16) / 16;  // image row of the 16-row tile
                    af[i] = *reinterpret_cast<const bf16x8_t *>(&sIn[((py + dy) * HW_ + l16 + dx) * LDK + kg * 8]);
                }
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    bfr[j] = *reinterpret_cast<const bf16x8_t *>(
                        &sW[(tap * BN + wn * (BN / 2) + j * 16 + l16) * LDK + kg * 8]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    if (KG > 1) {
        // partial tiles of groups 1 .. KG-1 into group 0's, in group order
        float *red = reinterpret_cast<float *>(smem);
        __syncthreads();
        if (grp > 0) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        red[(((grp - 1) * TM * TN + i * TN + j) * 4 + r) * 256 + tid] = acc[i][j][r];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int g = 1; g < KG; ++g)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            acc[i][j][r] += red[(((g - 1) * TM * TN + i * TN + j) * 4 + r) * 256 + tid];
        }
    }

    // D layout: tile row 4 (lane / 16) + r = pixel x0 + 4 kg + r of image
    // row y0 + py; column lane % 16.  Group 0 stores.
    __shared__ float fsum[2][MT];
    if (grp == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int pl = wm * (MT / 2) + i * 16;
            const int yy = y0 + pl / 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int xx = x0 + kg * 4 + r;
                const bool mok = yy < H && xx < W;
                const size_t m = ((size_t)b * H + yy) * W + xx;
                float f = 0.f;
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int n = n0 + wn * (BN / 2) + j * 16 + l16;
                    float v = acc[i][j][r] + bcol[j];
                    if (a.relu) v = fmaxf(v, 0.f);
                    const bf16_t h = f2bf(v);
                    if (mok && n < a.Nw) a.out[m * a.out_cs + a.out_co + n] = h;
                    f += bf2f(h) * fwc[j];
                }
                if (a.mode == 3) {
#pragma unroll
                    for (int o = 1; o < 16; o <<= 1) f += __shfl_xor(f, o, 16);
                    if (l16 == 0) fsum[wn][pl + kg * 4 + r] = f;
                }
            }
        }
    }
    if (a.mode == 3) {
        __syncthreads();
        if (threadIdx.x < MT) {
            const int yy = y0 + threadIdx.x / 16, xx = x0 + threadIdx.x % 16;
            if (yy < H && xx < W)
                a.out32[((size_t)b * H + yy) * W + xx] =
                    a.oscale * (fsum[0][threadIdx.x] + fsum[1][threadIdx.x] + a.fb[0]);
        }
    }
}

// First layer (3x3, one fed input channel): a thread computes 8 output
// channels of one pixel as FP32 sums over the nine taps of the BF16-rounded
// scaled input times the BF16 weights, then bias, ReLU and the BF16 NHWC
// store (a.in32 FP32 [B][H][W], weights w[t][n][Cin] with channel 0 fed).
__global__ void __launch_bounds__(256) k_conv_first(ConvArgs a)
{
    // the fed channel's weights of every tap and column, as FP32 in LDS
    __shared__ float sw[9 * 128];
    for (int k = threadIdx.x; k < 9 * a.Nw; k += blockDim.x) sw[k] = bf2f(a.w[(size_t)k * a.Cin]);
    __syncthreads();
    const int ng = a.Nw / 8;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long npix = (long long)a.B * a.Hout * a.Wout;
    if (i >= npix * ng) return;
    const int grp = (int)(i % ng);
    const long long p = i / ng;
    const int HW = a.Hout * a.Wout;
    const int b = (int)(p / HW), r = (int)(p - (long long)b * HW), oh = r / a.Wout, ow = r - oh * a.Wout;
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ih = oh + t / 3 - 1, iw = ow + t % 3 - 1;
        if (ih < 0 || ih >= a.Hin || iw < 0 || iw >= a.Win) continue;
        const float xv = bf2f(f2bf(a.in32[((size_t)b * a.Hin + ih) * a.Win + iw] * a.in_scale));
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = fmaf(xv, sw[t * a.Nw + grp * 8 + k], acc[k]);
    }
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        float v0 = acc[k] + a.bias[grp * 8 + k], v1 = acc[k + 1] + a.bias[grp * 8 + k + 1];
        if (a.relu) {
            v0 = fmaxf(v0, 0.f);
            v1 = fmaxf(v1, 0.f);
        }
        o[k / 2] = (uint32_t)f2bf(v0) | ((uint32_t)f2bf(v1) << 16);
    }
    *reinterpret_cast<uint4 *>(a.out + (size_t)p * a.out_cs + a.out_co + grp * 8) = make_uint4(o[0], o[1], o[2], o[3]);
}

// sum of the split-K partials in z order (a fixed order), then the epilogue
__global__ void __launch_bounds__(256) k_conv_splitk(ConvArgs a, int nz, const float *part)
{
    const size_t M = (size_t)a.B * a.Hout * a.Wout;
    const size_t len = M * a.Nw;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int z = 0; z < nz; ++z) v += part[(size_t)z * len + i];
        const int m = (int)(i / a.Nw), n = (int)(i - (size_t)m * a.Nw);
        conv_store(a, m, n, v, conv_bias(a, n));
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[t][n][c] = sum_m dY(m)[n] X(pix(m, t))[c], K-split
// over pixel chunks; partial tiles to part[chunk][t][n][c] (FP32).
// dY is either NHWC over the GEMM row grid (mode 0) or, for a transposed
// convolution (mode 2), gathered from the 2x up-sampled grid with
// n = (2a + b) cout + co.  Block: 4 waves, wave w owns c-tile 4 y + w.
// ---------------------------------------------------------------------------
struct WgradArgs {
    const bf16_t *x;
    int x_cs, x_co, Hin, Win, Cin;
    int ntaps, tw, org, stride;
    const bf16_t *dy;
    int dy_cs, dy_co, Nw, mode, cout;
    int B, Hout, Wout;
    int chunk;
    float *part;
};

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HWo = a.Hout * a.Wout, M = a.B * HWo;
    const int n0 = blockIdx.x * 16;
    const int c0 = (blockIdx.y * 4 + wave) * 16;
    const int t = blockIdx.z % a.ntaps;
    const int ch = blockIdx.z / a.ntaps;
    const int mbeg = ch * a.chunk, mend = min(M, mbeg + a.chunk);
    const int th = t / a.tw + a.org, twd = t % a.tw + a.org;
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
    const int n = n0 + (lane & 15), c = c0 + (lane & 15);
    const bool nok = n < a.Nw, cok = c < a.Cin;
    for (int m0 = mbeg; m0 < mend; m0 += 16) {
        short4_t av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + (lane >> 4) * 4 + j;
            short va = 0, vb = 0;
            if (m < mend) {
                const int bb = m / HWo, rr = m - bb * HWo, oh = rr / a.Wout, ow = rr - oh * a.Wout;
                if (nok) {
                    if (a.mode == 0) {
                        va = (short)a.dy[(size_t)m * a.dy_cs + a.dy_co + n];
                    } else {
                        const int ab = n / a.cout, co = n - ab * a.cout;
                        const size_t pix = ((size_t)bb * (2 * a.Hout) + 2 * oh + (ab >> 1)) * (2 * a.Wout) +
                                           2 * ow + (ab & 1);
                        va = (short)a.dy[pix * a.dy_cs + a.dy_co + co];
                    }
                }
                const int ih = oh * a.stride + th, iw = ow * a.stride + twd;
                if (cok && ih >= 0 && ih < a.Hin && iw >= 0 && iw < a.Win)
                    vb = (short)a.x[((size_t)(bb * a.Hin + ih) * a.Win + iw) * a.x_cs + a.x_co + c];
            }
            av[j] = va;
            bv[j] = vb;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    // D[i = n-row][col = c]: lane holds col = lane % 16, row = 4 (lane / 16) + j
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int nn = n0 + (lane >> 4) * 4 + j;
        if (nn < a.Nw && cok)
            a.part[(((size_t)ch * a.ntaps + t) * a.Nw + nn) * a.Cin + c] = acc[j];
    }
}

// LDS-staged weight gradient for Nw and Cin multiples of 8 (every layer but
// the one-column final): block tile 64 (n) x 64 (c) of one tap, K = pixels
// of the block's chunk in steps of 32.  Each thread loads 8 channels of one
// pixel of dY and of X (16 bytes each) and stores them transposed
// ([channel][pixel]) so that MFMA fragments are 16-byte LDS reads; 4 steps
// are staged per barrier.  Chunk lengths are multiples of 32.
__global__ void __launch_bounds__(256) k_wgrad2(WgradArgs a)
{
    constexpr int LDK = 40;
    constexpr int KC = 4;  // 32-pixel steps staged per barrier
    __shared__ __attribute__((aligned(16))) bf16_t sA[KC][64 * LDK];
    __shared__ __attribute__((aligned(16))) bf16_t sB[KC][64 * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int HWo = a.Hout * a.Wout, M = a.B * HWo;
    const int n0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    const int t = blockIdx.z % a.ntaps, ch = blockIdx.z / a.ntaps;
    const int mbeg = ch * a.chunk, mend = min(M, mbeg + a.chunk);
    const int th = t / a.tw + a.org, twd = t % a.tw + a.org;
    const int p = tid >> 3, cg = tid & 7;
    const int nA = n0 + 8 * cg, cB = c0 + 8 * cg;
    const bool nok = nA < a.Nw, cok = cB < a.Cin;
    int ab = 0, co = nA;
    if (a.mode == 2 && nok) {
        ab = nA / a.cout;
        co = nA - ab * a.cout;
    }
    // pixel of this thread in the next step to load: m = m0 + p, decoded incrementally
    int m = mbeg + p;
    int bb = 0, oh = 0, ow = 0;
    {
        const int mm = min(m, M - 1);
        bb = mm / HWo;
        const int r = mm - bb * HWo;
        oh = r / a.Wout;
        ow = r - oh * a.Wout;
    }
    uint4 va[KC], vb[KC];
    auto gload = [&]() {
#pragma unroll
        for (int s = 0; s < KC; ++s) {
            va[s] = make_uint4(0, 0, 0, 0);
            vb[s] = va[s];
            if (m < mend) {
                if (nok) {
                    size_t off;
                    if (a.mode == 0)
                        off = (size_t)m * a.dy_cs + a.dy_co + nA;
                    else
                        off = (((size_t)bb * (2 * a.Hout) + 2 * oh + (ab >> 1)) * (2 * a.Wout) + 2 * ow + (ab & 1)) *
                                  a.dy_cs + a.dy_co + co;
                    va[s] = *reinterpret_cast<const uint4 *>(a.dy + off);
                }
                const int ih = oh * a.stride + th, iw = ow * a.stride + twd;
                if (cok && ih >= 0 && ih < a.Hin && iw >= 0 && iw < a.Win)
                    vb[s] = *reinterpret_cast<const uint4 *>(a.x + ((size_t)(bb * a.Hin + ih) * a.Win + iw) * a.x_cs +
                                                             a.x_co + cB);
            }
            m += 32;
            ow += 32;
            while (ow >= a.Wout) {
                ow -= a.Wout;
                if (++oh == a.Hout) {
                    oh = 0;
                    ++bb;
                }
            }
        }
    };
    float4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    if (mbeg < mend) gload();
    for (int m0 = mbeg; m0 < mend; m0 += 32 * KC) {
        if (m0 != mbeg) __syncthreads();
#pragma unroll
        for (int s = 0; s < KC; ++s) {
            const bf16_t *ea = reinterpret_cast<const bf16_t *>(&va[s]);
            const bf16_t *eb = reinterpret_cast<const bf16_t *>(&vb[s]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sA[s][(8 * cg + j) * LDK + p] = ea[j];
                sB[s][(8 * cg + j) * LDK + p] = eb[j];
            }
        }
        __syncthreads();
        if (m0 + 32 * KC < mend) gload();
        const int ns = min(KC, (mend - m0 + 31) / 32);
#pragma unroll
        for (int s = 0; s < KC; ++s) {
            if (s >= ns) break;
            bf16x8_t af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                af[i] = *reinterpret_cast<const bf16x8_t *>(
                    &sA[s][(wm * 32 + i * 16 + (lane & 15)) * LDK + (lane >> 4) * 8]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8_t *>(
                    &sB[s][(wn * 32 + j * 16 + (lane & 15)) * LDK + (lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = c0 + wn * 32 + j * 16 + (lane & 15);
            if (c >= a.Cin) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = n0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
                if (n < a.Nw) a.part[(((size_t)ch * a.ntaps + t) * a.Nw + n) * a.Cin + c] = acc[i][j][r];
            }
        }
}

// out[i] = sum over c < nch of part[c][i], for i < len.  A block covers
// 256 / G consecutive i with G groups of threads; group q sums chunks
// q, q + G, ... in order, and the G group sums are added in order: a fixed
// order for a given (nch, G), with loads coalesced along i.
template <int G>
__global__ void __launch_bounds__(256) k_sum_chunks(const float *part, int nch, size_t len, float *out)
{
    constexpr int E = 256 / G;
    __shared__ float red[G][E];
    const int e = threadIdx.x % E, q = threadIdx.x / E;
    const size_t i = (size_t)blockIdx.x * E + e;
    float s = 0.f;
    if (i < len)
        for (int c = q; c < nch; c += G) s += part[(size_t)c * len + i];
    red[q][e] = s;
    __syncthreads();
    if (q == 0 && i < len) {
        float v = red[0][e];
#pragma unroll
        for (int k = 1; k < G; ++k) v += red[k][e];
        out[i] = v;
    }
}

// bias gradient partials: part[b][n] = sum over pixels p in block b's chunk
// of dy[p][dy_co + n], n < C.  Threads take 8 consecutive channels of one
// pixel (C a multiple of 8) or one channel (otherwise); the pixel lanes of a
// block are summed in order through LDS.
__global__ void __launch_bounds__(256)
k_bias_partial(const bf16_t *dy, int dy_cs, int dy_co, int C, int npix, int chunk, float *part)
{
    __shared__ float red[256 * 8];
    const int p0 = blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    const bool vec = C % 8 == 0 && C <= 2048;
    const int cpt = vec ? 8 : 1;
    const int groups = vec ? C / 8 : C;  // threads per pixel
    const int lanes = groups <= 256 ? 256 / groups : 1;
    const int gi = threadIdx.x % groups, pl = threadIdx.x / groups;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (groups <= 256 && pl < lanes) {
        for (int p = p0 + pl; p < p1; p += lanes) {
            const bf16_t *src = dy + (size_t)p * dy_cs + dy_co + gi * cpt;
            if (vec) {
                const uint4 v = *reinterpret_cast<const uint4 *>(src);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[2 * j] += bf2f((bf16_t)(w[j] & 0xffff));
                    acc[2 * j + 1] += bf2f((bf16_t)(w[j] >> 16));
                }
            } else {
                acc[0] += bf2f(*src);
            }
        }
    }
    for (int j = 0; j < cpt; ++j) red[threadIdx.x * 8 + j] = acc[j];
    __syncthreads();
    // thread k < C: channel k = group k / cpt, element k % cpt; sum lanes in order
    for (int k = threadIdx.x; k < C && groups <= 256; k += blockDim.x) {
        const int gk = k / cpt, jk = k - gk * cpt;
        float v = 0.f;
        for (int l = 0; l < lanes; ++l) v += red[(l * groups + gk) * 8 + jk];
        part[(size_t)blockIdx.x * C + k] = v;
    }
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
// input [B][H][W] FP32 * scale -> BF16 NHWC with 16 channels (channel 0 data)
__global__ void k_prep_input(const float *x, float scale, int npix, bf16_t *out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    out[(size_t)p * 16] = f2bf(x[p] * scale);
#pragma unroll
    for (int c = 1; c < 16; ++c) out[(size_t)p * 16 + c] = 0;
}

// dz = dy * (y > 0) on channel windows (in place on dy)
__global__ void k_relu_bwd(bf16_t *dy, int dy_cs, int dy_co, const bf16_t *y, int y_cs, int y_co,
                           int C, size_t npix)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C) return;
    const size_t p = i / C;
    const int c = (int)(i - p * C);
    if (!(bf2f(y[p * y_cs + y_co + c]) > 0.f)) dy[p * dy_cs + dy_co + c] = 0;
}

__global__ void k_maxpool(const bf16_t *in, int in_cs, int in_co, int B, int H, int W, int C,
                          bf16_t *out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (i >= (size_t)B * Ho * Wo * C) return;
    const int c = (int)(i % C);
    size_t r = i / C;
    const int ow = (int)(r % Wo);
    r /= Wo;
    const int oh = (int)(r % Ho);
    const int b = (int)(r / Ho);
    float m = -INFINITY;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const size_t pix = ((size_t)b * H + 2 * oh + (a >> 1)) * W + 2 * ow + (a & 1);
        m = fmaxf(m, bf2f(in[pix * in_cs + in_co + c]));
    }
    out[i] = f2bf(m);
}

// gradient to the first maximal element of each 2x2 window, ADDED to gin
__global__ void k_maxpool_bwd(const bf16_t *in, int in_cs, int in_co, int B, int H, int W, int C,
                              const bf16_t *gout, bf16_t *gin, int g_cs, int g_co)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (i >= (size_t)B * Ho * Wo * C) return;
    const int c = (int)(i % C);
    size_t r = i / C;
    const int ow = (int)(r % Wo);
    r /= Wo;
    const int oh = (int)(r % Ho);
    const int b = (int)(r / Ho);
    float m = -INFINITY;
    int arg = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const size_t pix = ((size_t)b * H + 2 * oh + (a >> 1)) * W + 2 * ow + (a & 1);
        const float v = bf2f(in[pix * in_cs + in_co + c]);
        if (v > m) {
            m = v;
            arg = a;
        }
    }
    const size_t pix = ((size_t)b * H + 2 * oh + (arg >> 1)) * W + 2 * ow + (arg & 1);
    bf16_t *g = gin + pix * g_cs + g_co + c;
    *g = f2bf(bf2f(*g) + bf2f(gout[i]));
}

// MSE loss: partial sums of (y - t)^2 per block; dy16[p][0] = gscale (y - t)
// (gscale = 2 oscale / npix: the gradient with respect to the last layer's
// pre-scale output)
__global__ void __launch_bounds__(256)
k_mse(const float *y, const float *t, int npix, float gscale, bf16_t *dy16, double *part)
{
    __shared__ double red[256];
    double s = 0.0;
    const float inv = gscale;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += gridDim.x * blockDim.x) {
        const float d = y[p] - t[p];
        s += (double)d * d;
        dy16[(size_t)p * 16] = f2bf(d * inv);
#pragma unroll
        for (int c = 1; c < 16; ++c) dy16[(size_t)p * 16 + c] = 0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x >> 1; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_fin(const double *part, int np, int npix, float *loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += part[i];
    *loss = (float)(s / npix);
}

// Adam on the flat FP32 parameters (Kingma & Ba, bias-corrected moments;
// c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t))
__global__ void k_adam(float *w, const float *g, float *m, float *v, size_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// BF16 copies: forward layout (same as master) and, for the data gradient,
// flipped / transposed wt[t'][c][n] = w[ntaps-1-t'][n][c] (3x3) or
// wt[t][c][n] = w[t][n][c] (2x2 transposed-convolution taps), with the n
// axis zero-padded to Np >= N.
__global__ void k_to_bf16(const float *w, size_t n, bf16_t *o)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = f2bf(w[i]);
}

__global__ void k_fill(float *p, size_t n, float v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_transpose_taps(const float *w, int ntaps, int N, int C, int Np, int flip, bf16_t *wt)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)ntaps * Np * C) return;
    const int n = (int)(i % Np);
    size_t r = i / Np;
    const int c = (int)(r % C);
    const int tp = (int)(r / C);
    const int t = flip ? ntaps - 1 - tp : tp;
    wt[i] = n < N ? f2bf(w[((size_t)t * N + n) * C + c]) : (bf16_t)0;
}

}  // namespace gct

// ---------------------------------------------------------------------------
// Host executor
// ---------------------------------------------------------------------------
namespace gct {
namespace {

enum { L_CONV = 0, L_UP = 1, L_FINAL = 2 };

struct ULayer {
    int kind;
    int ntaps, tw, org, stride;  // forward gather geometry
    int Cin, Nw, cout;           // weight [ntaps][Nw][Cin], bias [cout]
    size_t w_off, b_off;         // flat FP32 master / BF16 copy
    size_t wt_off;               // transposed BF16 copy for the data gradient
    bool need_dgrad;
};

inline size_t al64(size_t n) { return (n + 63) & ~(size_t)63; }
inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// K-split of a weight gradient over M GEMM rows: about 1024 blocks in all.
// nch never exceeds wgrad_max_chunks(L, M') for any M' >= M.
inline bool wgrad_tiled(const ULayer &L) { return L.Nw % 8 == 0 && L.Cin % 8 == 0; }

long long wgrad_max_chunks(const ULayer &L, long long M)
{
    const long long tiles = (long long)(wgrad_tiled(L) ? cdiv(L.Nw, 64) : cdiv(L.Nw, 16)) * cdiv(L.Cin, 64) * L.ntaps;
    const long long len = (long long)L.ntaps * L.Nw * L.Cin;
    long long n = std::min((1024 + tiles - 1) / tiles, (M + 255) / 256);
    n = std::min(n, (4LL << 20) / len);  // partials at most 4 Mi floats
    return std::max(1LL, n);
}

void wgrad_split(const ULayer &L, long long M, int &nch, int &chunk)
{
    const long long n = wgrad_max_chunks(L, M);
    long long c = (M + n - 1) / n;
    c = (c + 31) & ~31LL;
    chunk = (int)c;
    nch = (int)((M + c - 1) / c);
}

void bias_split(long long npix, int &nblk, int &chunk)
{
    long long c = std::max(256LL, (npix + 511) / 512);
    chunk = (int)c;
    nblk = (int)((npix + c - 1) / c);
}

}  // namespace
}  // namespace gct

struct gct_unet {
    int L, C0, H, W, maxB, device;
    std::vector<gct::ULayer> layers;
    std::vector<int> enc1, enc2, up, dec1, dec2;
    int fin;
    size_t nparam, nwt;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    gct::bf16_t *w16 = nullptr, *wt16 = nullptr;
    float *part = nullptr;
    size_t part_elems;
    double *lpart = nullptr;
    float *loss = nullptr;
    // activations and their gradients, per level
    std::vector<gct::bf16_t *> x, e, s, d1, d2, gx, ge, gs, gd1, gd2;
    gct::bf16_t *dy16 = nullptr;
    void *arena = nullptr;
    float oscale = 1.f;
    int last_batch = 0;
    // input of the last forward (the backward rebuilds the prepared input)
    const float *fx = nullptr;
    float fscale = 1.f;
    // captured forwards, keyed by their arguments (the other buffers are the
    // net's own), and the private stream they are captured on
    struct FwdGraph {
        int B;
        const float *x;
        float *y;
        float in_scale, out_scale;
        hipGraphExec_t exec;
    };
    std::vector<FwdGraph> fgraphs;
    hipStream_t capture = nullptr;

    int C(int l) const { return C0 << l; }
    int Hl(int l) const { return H >> l; }
    int Wl(int l) const { return W >> l; }
};

namespace gct {
namespace {

hipError_t last_launch() { return hipGetLastError(); }

// Tile shape and K split of the LDS-tiled convolution for an M x Nw x K
// GEMM: BN = 32 for narrow outputs, BM = 128 when that still gives >= 512
// blocks (two per CU); K is split where few blocks run long chains (below).
struct ConvTiling {
    int BM, BN, ksplit, steps;
};

ConvTiling conv_tiling(long long M, int Nw, int K)
{
    ConvTiling t;
    t.BN = Nw <= 32 ? 32 : 64;
    const long long nb = cdiv(Nw, t.BN);
    t.BM = (long long)cdiv(M, 128) * nb >= 512 ? 128 : 64;
    long long blocks = (long long)cdiv(M, t.BM) * nb;
    if (blocks < 256 && t.BN == 64) {  // narrower tiles before a K split
        t.BN = 32;
        blocks *= 2;
    }
    // K is split only where few blocks each run a long chain of 4-step
    // chunks: the split costs a reduce launch, worth it only when it removes
    // several dependent chunks per block; every part keeps >= 2 chunks
    const int nks = (K + 31) / 32, chunks = (nks + 3) / 4;
    int ks = 1;
    if (blocks < 256 && chunks > 4)
        ks = (int)std::min<long long>({16LL, (256 + blocks - 1) / blocks, (long long)chunks / 2});
    t.steps = (nks + ks - 1) / ks;
    t.ksplit = (nks + t.steps - 1) / t.steps;
    return t;
}

// FP32 elements of split-K partials a convolution needs (0 without a split)
size_t conv_part_elems(long long M, int Nw, int K)
{
    const ConvTiling t = conv_tiling(M, Nw, K);
    return t.ksplit > 1 ? (size_t)t.ksplit * M * Nw : 0;
}

// Tiles of the halo-tiled 3x3 kernel: 8 x 16 pixel tiles while they still
// give >= 256 blocks, else 4 x 16.  Short grids share the 32-channel chunks
// among wave groups: 4 groups below 256 blocks with >= 4 chunks (with
// 32-column tiles, which keeps the LDS of the block within 160 KB), else 2
// below 256 blocks or with >= 4 chunks below 512.  A pooled gather holds
// four times the input registers and takes at most 2 groups (the 128
// registers of a 1024-thread block would spill).
struct Conv33Tiling {
    int TY, BN, KG;
};

Conv33Tiling conv33_tiling(int B, int H, int W, int Nw, int Cin, bool pooled)
{
    Conv33Tiling t;
    t.BN = Nw <= 32 ? 32 : 64;
    const long long tiles8 = (long long)B * cdiv(H, 8) * cdiv(W, 16);
    t.TY = tiles8 * cdiv(Nw, t.BN) >= 256 ? 8 : 4;
    const long long blocks = (long long)B * cdiv(H, t.TY) * cdiv(W, 16) * cdiv(Nw, t.BN);
    const int nch = Cin / 32;
    t.KG = 1;
    if (blocks < 256 && nch >= 4 && !pooled) {
        t.KG = 4;
        t.BN = 32;
    } else if ((blocks < 256 && nch >= 2) || (blocks < 512 && nch >= 4)) {
        t.KG = 2;
    }
    return t;
}

bool conv33_ok(const ConvArgs &a, int in_kind)
{
    return a.ntaps == 9 && a.tw == 3 && a.org == -1 && a.stride == 1 && a.Cin % 32 == 0 && in_kind != 2 &&
           a.Hin == a.Hout && a.Win == a.Wout && (a.mode == 0 || a.mode == 3);
}


// in_kind: the input gather of k_conv2 (0 plain, 1 pooled, 2 FP32 first
// layer).  Pooled gathers hold four loads per A chunk, so they take the
// 64-row tile; mode 3 (fused final layer) is never K-split.
void conv_launch(const ConvArgs &a, hipStream_t st, float *part, int in_kind = 0)
{
    const long long M = (long long)a.B * a.Hout * a.Wout;
    if (a.mode == 1) {  // one output column: the plain kernel
        dim3 grid(cdiv(M, 64), cdiv(a.Nw, 64));
        hipLaunchKernelGGL(k_conv, grid, dim3(256), 0, st, a);
        return;
    }
    if (conv33_ok(a, in_kind)) {
        const Conv33Tiling t = conv33_tiling(a.B, a.Hout, a.Wout, a.Nw, a.Cin, in_kind == 1);
        dim3 grid((unsigned)((long long)a.B * cdiv(a.Hout, t.TY) * cdiv(a.Wout, 16)), cdiv(a.Nw, t.BN));
#define GCT_CONV33(TY_, BN_, IN_, KG_)                                                                      \
    if (t.TY == TY_ && t.BN == BN_ && in_kind == IN_ && t.KG == KG_) {                                      \
        hipLaunchKernelGGL((k_conv33<TY_, BN_, IN_, KG_>), grid, dim3(256 * KG_), 0, st, a);                \
        return;                                                                                             \
    }
        // (grouped K only below 256 blocks, where the tiles are 4 x 16)
        GCT_CONV33(8, 32, 0, 1) GCT_CONV33(8, 64, 0, 1) GCT_CONV33(4, 32, 0, 1) GCT_CONV33(4, 64, 0, 1)
        GCT_CONV33(4, 32, 0, 2) GCT_CONV33(4, 64, 0, 2) GCT_CONV33(4, 32, 0, 4)
        GCT_CONV33(8, 32, 1, 1) GCT_CONV33(8, 64, 1, 1) GCT_CONV33(4, 32, 1, 1) GCT_CONV33(4, 64, 1, 1)
        GCT_CONV33(4, 32, 1, 2) GCT_CONV33(4, 64, 1, 2)
#undef GCT_CONV33
    }
    if (in_kind == 2 && a.ntaps == 9 && a.mode == 0 && a.Nw % 8 == 0 && a.Nw <= 128 && a.out_co % 8 == 0 &&
        a.out_cs % 8 == 0) {
        const long long n = M * (a.Nw / 8);
        hipLaunchKernelGGL(k_conv_first, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, a);
        return;
    }
    ConvTiling t = conv_tiling(M, a.Nw, a.ntaps * a.Cin);
    if (in_kind == 1) t.BM = 64;
    if (a.mode == 3) {  // every column in the block, no K split
        t.BN = a.Nw <= 32 ? 32 : 64;
        t.steps = (a.ntaps * a.Cin + 31) / 32;
        t.ksplit = 1;
    }
    dim3 grid(cdiv(M, t.BM), cdiv(a.Nw, t.BN), t.ksplit);
#define GCT_CONV2(BM_, BN_, IN_) \
    hipLaunchKernelGGL((k_conv2<BM_, BN_, IN_>), grid, dim3(256), 0, st, a, t.steps, part)
    if (in_kind == 1) {
        if (t.BN == 64)
            GCT_CONV2(64, 64, 1);
        else
            GCT_CONV2(64, 32, 1);
    } else if (in_kind == 2) {
        if (t.BM == 128 && t.BN == 64)
            GCT_CONV2(128, 64, 2);
        else if (t.BM == 128)
            GCT_CONV2(128, 32, 2);
        else if (t.BN == 64)
            GCT_CONV2(64, 64, 2);
        else
            GCT_CONV2(64, 32, 2);
    } else {
        if (t.BM == 128 && t.BN == 64)
            GCT_CONV2(128, 64, 0);
        else if (t.BM == 128)
            GCT_CONV2(128, 32, 0);
        else if (t.BN == 64)
            GCT_CONV2(64, 64, 0);
        else
            GCT_CONV2(64, 32, 0);
    }
#undef GCT_CONV2
    if (t.ksplit > 1) {
        const long long len = M * a.Nw;
        hipLaunchKernelGGL(k_conv_splitk, dim3((unsigned)std::min<long long>(2048, cdiv(len, 256))), dim3(256), 0,
                           st, a, t.ksplit, (const float *)part);
    }
}

// forward of layer Lr: rows over the Hout x Wout grid (in_kind: see
// conv_launch; mode 3 fuses the final 1x1 layer and writes out32).  Hin x
// Win is the layer's input grid (pooled when in_kind = 1).
void fwd(const gct_unet *u, const ULayer &Lr, int B, const bf16_t *in, int in_cs, int in_co, int Hin,
         int Win, int Hout, int Wout, bf16_t *out, int out_cs, int out_co, int relu, int mode, float *out32,
         hipStream_t st, int in_kind = 0, const float *in32 = nullptr, float in_scale = 1.f)
{
    ConvArgs a{};
    a.in = in;
    a.in_cs = in_cs;
    a.in_co = in_co;
    a.B = B;
    a.Hin = Hin;
    a.Win = Win;
    a.Cin = Lr.Cin;
    a.ntaps = Lr.ntaps;
    a.tw = Lr.tw;
    a.org = Lr.org;
    a.stride = Lr.stride;
    a.w = u->w16 + Lr.w_off;
    a.Nw = Lr.Nw;
    a.Hout = Hout;
    a.Wout = Wout;
    a.bias = u->w + Lr.b_off;
    a.relu = relu;
    a.mode = mode;
    a.out = out;
    a.out_cs = out_cs;
    a.out_co = out_co;
    a.out32 = out32;
    a.oscale = u->oscale;
    a.cout = Lr.cout;
    a.in32 = in32;
    a.in_scale = in_scale;
    if (mode == 3) {
        const ULayer &F = u->layers[u->fin];
        a.fw = u->w16 + F.w_off;
        a.fb = u->w + F.b_off;
    }
    conv_launch(a, st, u->part, in_kind);
}

// data gradient of layer Lr: gin (rows over the layer's input grid) from
// gout (the layer's output gradient)
void dgrad(const gct_unet *u, const ULayer &Lr, int B, const bf16_t *gout, int go_cs, int go_co, int Hgo,
           int Wgo, int Hin, int Win, bf16_t *gin, int gi_cs, int gi_co, hipStream_t st)
{
    ConvArgs a{};
    a.in = gout;
    a.in_cs = go_cs;
    a.in_co = go_co;
    a.B = B;
    a.Hin = Hgo;
    a.Win = Wgo;
    a.w = u->wt16 + Lr.wt_off;
    a.Hout = Hin;
    a.Wout = Win;
    a.bias = nullptr;
    a.relu = 0;
    a.mode = 0;
    a.out = gin;
    a.out_cs = gi_cs;
    a.out_co = gi_co;
    a.oscale = 1.f;
    if (Lr.kind == L_CONV) {
        a.Cin = Lr.Nw;
        a.Nw = Lr.Cin;
        a.ntaps = 9;
        a.tw = 3;
        a.org = -1;
        a.stride = 1;
    } else if (Lr.kind == L_UP) {
        a.Cin = Lr.cout;
        a.Nw = Lr.Cin;
        a.ntaps = 4;
        a.tw = 2;
        a.org = 0;
        a.stride = 2;
    } else {
        a.Cin = 16;
        a.Nw = Lr.Cin;
        a.ntaps = 1;
        a.tw = 1;
        a.org = 0;
        a.stride = 1;
    }
    a.cout = a.Nw;
    conv_launch(a, st, u->part);
}

void sum_chunks(const float *part, int nch, size_t len, float *out, hipStream_t st)
{
    if (nch >= 16)
        hipLaunchKernelGGL(k_sum_chunks<16>, dim3(cdiv((long long)len, 16)), dim3(256), 0, st, part, nch, len, out);
    else if (nch >= 4)
        hipLaunchKernelGGL(k_sum_chunks<4>, dim3(cdiv((long long)len, 64)), dim3(256), 0, st, part, nch, len, out);
    else
        hipLaunchKernelGGL(k_sum_chunks<1>, dim3(cdiv((long long)len, 256)), dim3(256), 0, st, part, nch, len, out);
}

// weight and bias gradients of layer Lr into u->g
void wgrad(gct_unet *u, const ULayer &Lr, int B, const bf16_t *x, int x_cs, int x_co, int Hin, int Win,
           const bf16_t *dy, int dy_cs, int dy_co, int Hout, int Wout, hipStream_t st)
{
    WgradArgs a{};
    a.x = x;
    a.x_cs = x_cs;
    a.x_co = x_co;
    a.Hin = Hin;
    a.Win = Win;
    a.Cin = Lr.Cin;
    a.ntaps = Lr.ntaps;
    a.tw = Lr.tw;
    a.org = Lr.org;
    a.stride = Lr.stride;
    a.dy = dy;
    a.dy_cs = dy_cs;
    a.dy_co = dy_co;
    a.Nw = Lr.Nw;
    a.mode = Lr.kind == L_UP ? 2 : 0;
    a.cout = Lr.cout;
    a.B = B;
    a.Hout = Hout;
    a.Wout = Wout;
    const long long M = (long long)B * Hout * Wout;
    int nch, chunk;
    wgrad_split(Lr, M, nch, chunk);
    a.chunk = chunk;
    a.part = u->part;
    if (wgrad_tiled(Lr)) {
        dim3 grid(cdiv(Lr.Nw, 64), cdiv(Lr.Cin, 64), Lr.ntaps * nch);
        hipLaunchKernelGGL(k_wgrad2, grid, dim3(256), 0, st, a);
    } else {
        dim3 grid(cdiv(Lr.Nw, 16), cdiv(Lr.Cin, 64), Lr.ntaps * nch);
        hipLaunchKernelGGL(k_wgrad, grid, dim3(256), 0, st, a);
    }
    const size_t len = (size_t)Lr.ntaps * Lr.Nw * Lr.Cin;
    sum_chunks(u->part, nch, len, u->g + Lr.w_off, st);
    // bias: over the pixels of the layer's output grid
    long long npix;
    int bcs = dy_cs, bco = dy_co;
    if (Lr.kind == L_UP)
        npix = 4LL * M;
    else
        npix = M;
    int nblk, bchunk;
    bias_split(npix, nblk, bchunk);
    hipLaunchKernelGGL(k_bias_partial, dim3(nblk), dim3(256), 0, st, dy, bcs, bco, Lr.cout, (int)npix, bchunk,
                       u->part);
    sum_chunks(u->part, nblk, (size_t)Lr.cout, u->g + Lr.b_off, st);
}

void relu_bwd(bf16_t *gy, int g_cs, int g_co, const bf16_t *y, int y_cs, int y_co, int C, long long npix,
              hipStream_t st)
{
    const long long n = npix * C;
    hipLaunchKernelGGL(k_relu_bwd, dim3(cdiv(n, 256)), dim3(256), 0, st, gy, g_cs, g_co, y, y_cs, y_co, C,
                       (size_t)npix);
}

void refresh_bf16(gct_unet *u, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(cdiv((long long)u->nparam, 256)), dim3(256), 0, st, (const float *)u->w,
                       u->nparam, u->w16);
    for (const ULayer &Lr : u->layers) {
        if (!Lr.need_dgrad) continue;
        int nt, N, Cc, Np, flip;
        if (Lr.kind == L_CONV) {
            nt = 9; N = Lr.Nw; Cc = Lr.Cin; Np = Lr.Nw; flip = 1;
        } else if (Lr.kind == L_UP) {
            nt = 4; N = Lr.cout; Cc = Lr.Cin; Np = Lr.cout; flip = 0;
        } else {
            nt = 1; N = 1; Cc = Lr.Cin; Np = 16; flip = 0;
        }
        const long long n = (long long)nt * Np * Cc;
        hipLaunchKernelGGL(k_transpose_taps, dim3(cdiv(n, 256)), dim3(256), 0, st, (const float *)(u->w + Lr.w_off),
                           nt, N, Cc, Np, flip, u->wt16 + Lr.wt_off);
    }
}

void fill(float *p, size_t n, float v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(std::min(2048, cdiv((long long)n, 256))), dim3(256), 0, st, p, n, v);
}

ULayer make_layer(int kind, int Cin, int cout)
{
    ULayer Lr{};
    Lr.kind = kind;
    Lr.Cin = Cin;
    Lr.cout = cout;
    if (kind == L_CONV) {
        Lr.ntaps = 9; Lr.tw = 3; Lr.org = -1; Lr.stride = 1; Lr.Nw = cout;
    } else if (kind == L_UP) {
        Lr.ntaps = 1; Lr.tw = 1; Lr.org = 0; Lr.stride = 1; Lr.Nw = 4 * cout;
    } else {
        Lr.ntaps = 1; Lr.tw = 1; Lr.org = 0; Lr.stride = 1; Lr.Nw = 1;
    }
    Lr.need_dgrad = true;
    return Lr;
}

}  // namespace
}  // namespace gct

using namespace gct;

extern "C" {

int gct_unet_create(const gct_unet_config *cfg, gct_unet **out)
{
    if (!cfg || !out) return fail(GCT_EINVAL, "NULL argument");
    *out = nullptr;
    const int L = cfg->levels, C0 = cfg->base_channels;
    if (L < 1 || L > 6) return fail(GCT_EINVAL, "levels must be in [1, 6]");
    if (C0 < 16 || C0 % 16 != 0 || ((long long)C0 << (L - 1)) > 1024)
        return fail(GCT_EINVAL, "base_channels must be a multiple of 16 with base_channels 2^(levels-1) <= 1024");
    const int div = 1 << (L - 1);
    if (cfg->height < div || cfg->width < div || cfg->height % div || cfg->width % div)
        return fail(GCT_EINVAL, "height and width must be positive multiples of 2^(levels-1)");
    if (cfg->max_batch < 1 || (long long)cfg->max_batch * cfg->height * cfg->width > (1LL << 28))
        return fail(GCT_EINVAL, "max_batch must be >= 1 with max_batch height width <= 2^28");

    gct_unet *u = new gct_unet();
    u->L = L;
    u->C0 = C0;
    u->H = cfg->height;
    u->W = cfg->width;
    u->maxB = cfg->max_batch;
    if (hipGetDevice(&u->device) != hipSuccess) {
        delete u;
        return fail(GCT_EHIP, "hipGetDevice failed");
    }
    // parameter layout
    auto add = [&](ULayer Lr) {
        u->layers.push_back(Lr);
        return (int)u->layers.size() - 1;
    };
    u->enc1.assign(L, -1);
    u->enc2.assign(L, -1);
    u->up.assign(L, -1);
    u->dec1.assign(L, -1);
    u->dec2.assign(L, -1);
    for (int l = 0; l < L; ++l) {
        u->enc1[l] = add(make_layer(L_CONV, l == 0 ? 16 : u->C(l - 1), u->C(l)));
        u->enc2[l] = add(make_layer(L_CONV, u->C(l), u->C(l)));
    }
    u->layers[u->enc1[0]].need_dgrad = false;
    for (int l = L - 2; l >= 0; --l) {
        u->up[l] = add(make_layer(L_UP, u->C(l + 1), u->C(l)));
        u->dec1[l] = add(make_layer(L_CONV, 2 * u->C(l), u->C(l)));
        u->dec2[l] = add(make_layer(L_CONV, u->C(l), u->C(l)));
    }
    u->fin = add(make_layer(L_FINAL, C0, 1));
    size_t off = 0, woff = 0;
    for (ULayer &Lr : u->layers) {
        Lr.w_off = off;
        off = al64(off + (size_t)Lr.ntaps * Lr.Nw * Lr.Cin);
        Lr.b_off = off;
        off = al64(off + Lr.cout);
        Lr.wt_off = woff;
        const int np = Lr.kind == L_FINAL ? 16 : Lr.Nw;
        if (Lr.need_dgrad) woff = al64(woff + (size_t)Lr.ntaps * np * Lr.Cin);
    }
    u->nparam = off;
    u->nwt = std::max<size_t>(woff, 64);
    // scratch for K-split partials: the largest need over layers at max_batch
    // (weight gradients) and over every batch size (split convolutions)
    size_t part = 512 * 1024;
    for (int B = 1; B <= u->maxB; ++B) {
        for (int l = 0; l < L; ++l) {
            const long long Ml = (long long)B * u->Hl(l) * u->Wl(l);
            for (int idx : {u->enc1[l], u->enc2[l], u->dec1[l], u->dec2[l]}) {
                if (idx < 0) continue;
                const ULayer &Lr = u->layers[idx];
                part = std::max(part, conv_part_elems(Ml, Lr.Nw, 9 * Lr.Cin));
                part = std::max(part, conv_part_elems(Ml, Lr.Cin, 9 * Lr.Nw));
            }
            if (u->up[l] >= 0) {
                const ULayer &Lr = u->layers[u->up[l]];
                const long long Mn = (long long)B * u->Hl(l + 1) * u->Wl(l + 1);
                part = std::max(part, conv_part_elems(Mn, Lr.Nw, Lr.Cin));
                part = std::max(part, conv_part_elems(Mn, Lr.Cin, 4 * Lr.cout));
            }
        }
        part = std::max(part, conv_part_elems((long long)B * u->H * u->W, C0, 16));
    }
    for (int l = 0; l < L; ++l) {
        auto need = [&](int idx, long long M) {
            if (idx < 0) return;
            const ULayer &Lr = u->layers[idx];
            part = std::max(part, (size_t)wgrad_max_chunks(Lr, M) * Lr.ntaps * Lr.Nw * Lr.Cin);
            int nb, bc;
            bias_split(Lr.kind == L_UP ? 4 * M : M, nb, bc);
            part = std::max(part, (size_t)nb * Lr.cout);
        };
        const long long Ml = (long long)u->maxB * u->Hl(l) * u->Wl(l);
        need(u->enc1[l], Ml);
        need(u->enc2[l], Ml);
        need(u->dec1[l], Ml);
        need(u->dec2[l], Ml);
        if (u->up[l] >= 0) need(u->up[l], (long long)u->maxB * u->Hl(l + 1) * u->Wl(l + 1));
    }
    {
        const ULayer &Lr = u->layers[u->fin];
        part = std::max(part, (size_t)wgrad_max_chunks(Lr, (long long)u->maxB * u->H * u->W) * Lr.Cin);
    }
    u->part_elems = part;

    // activation arena
    std::vector<std::pair<gct::bf16_t **, size_t>> plan;
    u->x.assign(L, nullptr);
    u->e.assign(L, nullptr);
    u->s.assign(L, nullptr);
    u->d1.assign(L, nullptr);
    u->d2.assign(L, nullptr);
    u->gx.assign(L, nullptr);
    u->ge.assign(L, nullptr);
    u->gs.assign(L, nullptr);
    u->gd1.assign(L, nullptr);
    u->gd2.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
        const size_t px = (size_t)u->maxB * u->Hl(l) * u->Wl(l);
        const int Cl = u->C(l);
        const int cs = l < L - 1 ? 2 * Cl : Cl;
        plan.push_back({&u->x[l], px * (l == 0 ? 16 : u->C(l - 1))});
        plan.push_back({&u->e[l], px * Cl});
        plan.push_back({&u->s[l], px * cs});
        plan.push_back({&u->ge[l], px * Cl});
        plan.push_back({&u->gs[l], px * cs});
        if (l > 0) plan.push_back({&u->gx[l], px * u->C(l - 1)});
        if (l < L - 1) {
            plan.push_back({&u->d1[l], px * Cl});
            plan.push_back({&u->d2[l], px * Cl});
            plan.push_back({&u->gd1[l], px * Cl});
            plan.push_back({&u->gd2[l], px * Cl});
        }
    }
    plan.push_back({&u->dy16, (size_t)u->maxB * u->H * u->W * 16});
    size_t bytes = 0;
    std::vector<size_t> offs;
    for (auto &pr : plan) {
        offs.push_back(bytes);
        bytes += align256(pr.second * sizeof(gct::bf16_t));
    }
    hipError_t e = hipSuccess;
    auto grab = [&](void **p, size_t b) {
        if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(b, 256));
    };
    grab((void **)&u->w, u->nparam * 4);
    grab((void **)&u->g, u->nparam * 4);
    grab((void **)&u->m, u->nparam * 4);
    grab((void **)&u->v, u->nparam * 4);
    grab((void **)&u->w16, u->nparam * 2);
    grab((void **)&u->wt16, u->nwt * 2);
    grab((void **)&u->part, u->part_elems * 4);
    grab((void **)&u->lpart, 1024 * 8);
    grab((void **)&u->loss, 256);
    grab(&u->arena, bytes);
    if (e != hipSuccess) {
        gct_unet_destroy(u);
        return fail(GCT_EHIP, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    for (size_t i = 0; i < plan.size(); ++i) *plan[i].first = (gct::bf16_t *)((char *)u->arena + offs[i]);
    fill(u->w, u->nparam, 0.f, nullptr);
    fill(u->g, u->nparam, 0.f, nullptr);
    fill(u->m, u->nparam, 0.f, nullptr);
    fill(u->v, u->nparam, 0.f, nullptr);
    refresh_bf16(u, nullptr);
    e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        gct_unet_destroy(u);
        return fail(GCT_EHIP, std::string("U-Net init failed: ") + hipGetErrorString(e));
    }
    *out = u;
    return GCT_OK;
}

int gct_unet_destroy(gct_unet *u)
{
    if (!u) return GCT_OK;
    for (auto &g : u->fgraphs) (void)hipGraphExecDestroy(g.exec);
    if (u->capture) (void)hipStreamDestroy(u->capture);
    (void)hipFree(u->w);
    (void)hipFree(u->g);
    (void)hipFree(u->m);
    (void)hipFree(u->v);
    (void)hipFree(u->w16);
    (void)hipFree(u->wt16);
    (void)hipFree(u->part);
    (void)hipFree(u->lpart);
    (void)hipFree(u->loss);
    (void)hipFree(u->arena);
    delete u;
    return GCT_OK;
}

int gct_unet_param_count(const gct_unet *u, int64_t *n)
{
    if (!u || !n) return fail(GCT_EINVAL, "NULL argument");
    *n = (int64_t)u->nparam;
    return GCT_OK;
}

int gct_unet_layer_count(const gct_unet *u, int32_t *n)
{
    if (!u || !n) return fail(GCT_EINVAL, "NULL argument");
    *n = (int32_t)u->layers.size();
    return GCT_OK;
}

int gct_unet_layer_info(const gct_unet *u, int32_t i, gct_unet_layer *info)
{
    if (!u || !info) return fail(GCT_EINVAL, "NULL argument");
    if (i < 0 || i >= (int32_t)u->layers.size()) return fail(GCT_EINVAL, "layer index out of range");
    const ULayer &Lr = u->layers[i];
    info->kind = Lr.kind;
    info->taps = Lr.kind == L_CONV ? 9 : Lr.kind == L_UP ? 4 : 1;
    info->in_channels = Lr.Cin;
    info->out_channels = Lr.cout;
    info->weight_offset = (int64_t)Lr.w_off;
    info->bias_offset = (int64_t)Lr.b_off;
    return GCT_OK;
}

int gct_unet_set_params(gct_unet *u, const float *params, void *stream)
{
    if (!u || !params) return fail(GCT_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(u->w, params, u->nparam * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return check_hip(e, "gct_unet_set_params");
    refresh_bf16(u, st);
    return check_hip(last_launch(), "gct_unet_set_params");
}

int gct_unet_get_params(const gct_unet *u, float *params, void *stream)
{
    if (!u || !params) return fail(GCT_EINVAL, "NULL argument");
    return check_hip(hipMemcpyAsync(params, u->w, u->nparam * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream),
                     "gct_unet_get_params");
}

int gct_unet_get_grads(const gct_unet *u, float *grads, void *stream)
{
    if (!u || !grads) return fail(GCT_EINVAL, "NULL argument");
    return check_hip(hipMemcpyAsync(grads, u->g, u->nparam * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream),
                     "gct_unet_get_grads");
}

int gct_unet_get_moments(const gct_unet *u, float *m, float *v, void *stream)
{
    if (!u || !m || !v) return fail(GCT_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(m, u->m, u->nparam * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(v, u->v, u->nparam * 4, hipMemcpyDeviceToDevice, st);
    return check_hip(e, "gct_unet_get_moments");
}

int gct_unet_set_moments(gct_unet *u, const float *m, const float *v, void *stream)
{
    if (!u) return fail(GCT_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (!m || !v) {
        if (m || v) return fail(GCT_EINVAL, "m and v must both be given or both be NULL");
        fill(u->m, u->nparam, 0.f, st);
        fill(u->v, u->nparam, 0.f, st);
        return check_hip(last_launch(), "gct_unet_set_moments");
    }
    hipError_t e = hipMemcpyAsync(u->m, m, u->nparam * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(u->v, v, u->nparam * 4, hipMemcpyDeviceToDevice, st);
    return check_hip(e, "gct_unet_set_moments");
}

}  // extern "C"

// The forward's launches (queued on st; captured by gct_unet_forward).
// Input preparation and max pooling are fused into the consuming
// convolutions and the final 1x1 layer into the last 3x3 one, so the
// prepared input x[0] and the pooled x[l] are not stored here
// (recompute_inputs rebuilds them for the backward).
static bool fuse_final(const gct_unet *u) { return u->C0 <= 64; }

static void forward_launches(gct_unet *u, int B, const float *x, float in_scale, float *y, hipStream_t st)
{
    const int L = u->L;
    const bool ff = fuse_final(u);
    for (int l = 0; l < L; ++l) {
        const int Hl = u->Hl(l), Wl = u->Wl(l), Cl = u->C(l);
        if (l == 0)
            fwd(u, u->layers[u->enc1[0]], B, nullptr, 16, 0, Hl, Wl, Hl, Wl, u->e[0], Cl, 0, 1, 0, nullptr, st, 2, x,
                in_scale);
        else
            fwd(u, u->layers[u->enc1[l]], B, u->s[l - 1], 2 * u->C(l - 1), u->C(l - 1), Hl, Wl, Hl, Wl, u->e[l], Cl,
                0, 1, 0, nullptr, st, 1);
        if (l < L - 1)
            fwd(u, u->layers[u->enc2[l]], B, u->e[l], Cl, 0, Hl, Wl, Hl, Wl, u->s[l], 2 * Cl, Cl, 1, 0, nullptr, st);
        else
            fwd(u, u->layers[u->enc2[l]], B, u->e[l], Cl, 0, Hl, Wl, Hl, Wl, u->s[l], Cl, 0, 1,
                (L == 1 && ff) ? 3 : 0, y, st);
    }
    const bf16_t *prev = u->s[L - 1];
    for (int l = L - 2; l >= 0; --l) {
        const int Hl = u->Hl(l), Wl = u->Wl(l), Cl = u->C(l);
        const int Hn = u->Hl(l + 1), Wn = u->Wl(l + 1);
        fwd(u, u->layers[u->up[l]], B, prev, u->C(l + 1), 0, Hn, Wn, Hn, Wn, u->s[l], 2 * Cl, 0, 0, 2, nullptr, st);
        fwd(u, u->layers[u->dec1[l]], B, u->s[l], 2 * Cl, 0, Hl, Wl, Hl, Wl, u->d1[l], Cl, 0, 1, 0, nullptr, st);
        fwd(u, u->layers[u->dec2[l]], B, u->d1[l], Cl, 0, Hl, Wl, Hl, Wl, u->d2[l], Cl, 0, 1,
            (l == 0 && ff) ? 3 : 0, y, st);
        prev = u->d2[l];
    }
    if (!ff) fwd(u, u->layers[u->fin], B, prev, u->C0, 0, u->H, u->W, u->H, u->W, nullptr, 0, 0, 0, 1, y, st);
}

// The layer inputs the fused forward did not store: the prepared input
// (from the forward's x and in_scale) and the pooled input of every level
// below the first.
static void recompute_inputs(gct_unet *u, int B, hipStream_t st)
{
    const long long npix = (long long)B * u->H * u->W;
    hipLaunchKernelGGL(k_prep_input, dim3(cdiv(npix, 256)), dim3(256), 0, st, u->fx, u->fscale, (int)npix, u->x[0]);
    for (int l = 0; l + 1 < u->L; ++l) {
        const int Hl = u->Hl(l), Wl = u->Wl(l), Cl = u->C(l);
        const long long n = (long long)B * (Hl / 2) * (Wl / 2) * Cl;
        hipLaunchKernelGGL(k_maxpool, dim3(cdiv(n, 256)), dim3(256), 0, st, (const bf16_t *)u->s[l], 2 * Cl, Cl, B,
                           Hl, Wl, Cl, u->x[l + 1]);
    }
}

extern "C" {

int gct_unet_forward(gct_unet *u, int32_t batch, const float *x, float in_scale, float out_scale, float *y,
                     void *stream)
{
    if (!u || !x || !y) return fail(GCT_EINVAL, "NULL argument");
    if (batch < 1 || batch > u->maxB) return fail(GCT_EINVAL, "batch must be in [1, max_batch]");
    if (!std::isfinite(in_scale) || !std::isfinite(out_scale))
        return fail(GCT_EINVAL, "scales must be finite");
    if (x == y) return fail(GCT_EINVAL, "y must not alias x");
    hipStream_t st = (hipStream_t)stream;
    u->oscale = out_scale;
    // the launch sequence is replayed as a captured graph (one capture per
    // argument set; up to 8 kept)
    hipGraphExec_t exec = nullptr;
    for (const auto &g : u->fgraphs)
        if (g.B == batch && g.x == x && g.y == y && g.in_scale == in_scale && g.out_scale == out_scale) exec = g.exec;
    if (!exec) {
        if (!u->capture && hipStreamCreateWithFlags(&u->capture, hipStreamNonBlocking) != hipSuccess) {
            u->capture = nullptr;
            return fail(GCT_EHIP, "cannot create the capture stream");
        }
        hipError_t e = hipStreamBeginCapture(u->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return check_hip(e, "gct_unet_forward capture");
        forward_launches(u, batch, x, in_scale, y, u->capture);
        hipError_t el = hipGetLastError();
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(u->capture, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return check_hip(el != hipSuccess ? el : e, "gct_unet_forward capture");
        }
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return check_hip(e, "gct_unet_forward instantiate");
        if (u->fgraphs.size() >= 8) {
            (void)hipGraphExecDestroy(u->fgraphs.front().exec);
            u->fgraphs.erase(u->fgraphs.begin());
        }
        u->fgraphs.push_back({batch, x, y, in_scale, out_scale, exec});
    }
    u->last_batch = batch;
    u->fx = x;
    u->fscale = in_scale;
    return check_hip(hipGraphLaunch(exec, st), "gct_unet_forward");
}

int gct_unet_backward(gct_unet *u, int32_t batch, const float *y, const float *target, float *loss,
                      void *stream)
{
    if (!u || !y || !target) return fail(GCT_EINVAL, "NULL argument");
    if (batch != u->last_batch) return fail(GCT_EINVAL, "batch differs from the preceding forward");
    hipStream_t st = (hipStream_t)stream;
    const int L = u->L, B = batch;
    const long long npix = (long long)B * u->H * u->W;
    const int nb = std::min(1024, cdiv(npix, 256));
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, y, target, (int)npix, 2.f * u->oscale / (float)npix,
                       u->dy16, u->lpart);
    hipLaunchKernelGGL(k_mse_fin, dim3(1), dim3(64), 0, st, (const double *)u->lpart, nb, (int)npix,
                       loss ? loss : u->loss);
    recompute_inputs(u, B, st);
    // final 1x1
    bf16_t *top = L > 1 ? u->d2[0] : u->s[0];
    bf16_t *gtop = L > 1 ? u->gd2[0] : u->gs[0];
    {
        const ULayer &Lr = u->layers[u->fin];
        wgrad(u, Lr, B, top, u->C0, 0, u->H, u->W, u->dy16, 16, 0, u->H, u->W, st);
        dgrad(u, Lr, B, u->dy16, 16, 0, u->H, u->W, u->H, u->W, gtop, u->C0, 0, st);
    }
    // decoder, top level first
    for (int l = 0; l <= L - 2; ++l) {
        const int Hl = u->Hl(l), Wl = u->Wl(l), Cl = u->C(l);
        const long long px = (long long)B * Hl * Wl;
        relu_bwd(u->gd2[l], Cl, 0, u->d2[l], Cl, 0, Cl, px, st);
        const ULayer &D2 = u->layers[u->dec2[l]];
        wgrad(u, D2, B, u->d1[l], Cl, 0, Hl, Wl, u->gd2[l], Cl, 0, Hl, Wl, st);
        dgrad(u, D2, B, u->gd2[l], Cl, 0, Hl, Wl, Hl, Wl, u->gd1[l], Cl, 0, st);
        relu_bwd(u->gd1[l], Cl, 0, u->d1[l], Cl, 0, Cl, px, st);
        const ULayer &D1 = u->layers[u->dec1[l]];
        wgrad(u, D1, B, u->s[l], 2 * Cl, 0, Hl, Wl, u->gd1[l], Cl, 0, Hl, Wl, st);
        dgrad(u, D1, B, u->gd1[l], Cl, 0, Hl, Wl, Hl, Wl, u->gs[l], 2 * Cl, 0, st);
        // transposed convolution from level l+1
        const int Hn = u->Hl(l + 1), Wn = u->Wl(l + 1), Cn = u->C(l + 1);
        const bool bott = l + 1 == L - 1;
        const bf16_t *pin = bott ? u->s[L - 1] : u->d2[l + 1];
        bf16_t *gpin = bott ? u->gs[L - 1] : u->gd2[l + 1];
        const ULayer &U = u->layers[u->up[l]];
        wgrad(u, U, B, pin, Cn, 0, Hn, Wn, u->gs[l], 2 * Cl, 0, Hn, Wn, st);
        dgrad(u, U, B, u->gs[l], 2 * Cl, 0, Hl, Wl, Hn, Wn, gpin, Cn, 0, st);
    }
    // bottleneck
    {
        const int l = L - 1, Hl = u->Hl(l), Wl = u->Wl(l), Cl = u->C(l);
        const long long px = (long long)B * Hl * Wl;
        relu_bwd(u->gs[l], Cl, 0, u->s[l], Cl, 0, Cl, px, st);
        const ULayer &E2 = u->layers[u->enc2[l]];
        wgrad(u, E2, B, u->e[l], Cl, 0, Hl, Wl, u->gs[l], Cl, 0, Hl, Wl, st);
        dgrad(u, E2, B, u->gs[l], Cl, 0, Hl, Wl, Hl, Wl, u->ge[l], Cl, 0, st);
        relu_bwd(u->ge[l], Cl, 0, u->e[l], Cl, 0, Cl, px, st);
        const ULayer &E1 = u->layers[u->enc1[l]];
        const int xc = l == 0 ? 16 : u->C(l - 1);
        wgrad(u, E1, B, u->x[l], xc, 0, Hl, Wl, u->ge[l], Cl, 0, Hl, Wl, st);
        if (l > 0) dgrad(u, E1, B, u->ge[l], Cl, 0, Hl, Wl, Hl, Wl, u->gx[l], xc, 0, st);
    }
    // encoder, deepest first
    for (int l = L - 2; l >= 0; --l) {
        const int Hl = u->Hl(l), Wl = u->Wl(l), Cl = u->C(l);
        const long long px = (long long)B * Hl * Wl;
        const long long n = (long long)B * (Hl / 2) * (Wl / 2) * Cl;
        hipLaunchKernelGGL(k_maxpool_bwd, dim3(cdiv(n, 256)), dim3(256), 0, st, (const bf16_t *)u->s[l], 2 * Cl, Cl,
                           B, Hl, Wl, Cl, (const bf16_t *)u->gx[l + 1], u->gs[l], 2 * Cl, Cl);
        relu_bwd(u->gs[l], 2 * Cl, Cl, u->s[l], 2 * Cl, Cl, Cl, px, st);
        const ULayer &E2 = u->layers[u->enc2[l]];
        wgrad(u, E2, B, u->e[l], Cl, 0, Hl, Wl, u->gs[l], 2 * Cl, Cl, Hl, Wl, st);
        dgrad(u, E2, B, u->gs[l], 2 * Cl, Cl, Hl, Wl, Hl, Wl, u->ge[l], Cl, 0, st);
        relu_bwd(u->ge[l], Cl, 0, u->e[l], Cl, 0, Cl, px, st);
        const ULayer &E1 = u->layers[u->enc1[l]];
        const int xc = l == 0 ? 16 : u->C(l - 1);
        wgrad(u, E1, B, u->x[l], xc, 0, Hl, Wl, u->ge[l], Cl, 0, Hl, Wl, st);
        if (l > 0) dgrad(u, E1, B, u->ge[l], Cl, 0, Hl, Wl, Hl, Wl, u->gx[l], xc, 0, st);
    }
    return check_hip(last_launch(), "gct_unet_backward");
}

int gct_unet_adam_step(gct_unet *u, float lr, float beta1, float beta2, float eps, int32_t step, void *stream)
{
    if (!u) return fail(GCT_EINVAL, "NULL argument");
    if (step < 1) return fail(GCT_EINVAL, "step counts from 1");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(GCT_EINVAL, "bad Adam hyper-parameters");
    hipStream_t st = (hipStream_t)stream;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    hipLaunchKernelGGL(k_adam, dim3(cdiv((long long)u->nparam, 256)), dim3(256), 0, st, u->w, (const float *)u->g,
                       u->m, u->v, u->nparam, lr, beta1, beta2, eps, c1, c2);
    refresh_bf16(u, st);
    return check_hip(last_launch(), "gct_unet_adam_step");
}

}  // extern "C"
