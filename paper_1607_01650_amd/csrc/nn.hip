// BF16 MFMA convolution kernels (gfx950) and the small kernels of the U-Net
// that maps an early ADM iterate to a late one (learned warm start).
//
// Tensors are NHWC, activations and weights BF16, accumulation FP32 on the
// matrix cores (v_mfma_f32_16x16x32_bf16).  Convolutions are implicit GEMMs:
//   forward / dgrad : D[pixel][co] = sum_k A[pixel][k] B[k][co], k = (tap, ci)
//   wgrad           : D[co][ci]    = sum_p dZ[p][co] X[p + tap][ci] per tap
// dgrad is the forward kernel run on dZ with taps flipped and channels
// transposed; a 2x2 stride-2 transposed convolution is a 1x1 convolution to
// 4*Cout channels followed by depth-to-space.  Every reduction that crosses
// blocks goes through per-block partials summed in a fixed order.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstdint>

#include "../../include/dect_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

thread_local const char *g_nn_err = "";

dect_status nn_fail(dect_status st, const char *msg)
{
    g_nn_err = msg;
    return st;
}

#define NN_HIP(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) return nn_fail(DECT_ERR_HIP, hipGetErrorString(e_)); \
    } while (0)

__device__ __forceinline__ float bf2f(u16 v) { return __uint_as_float((uint32_t)v << 16); }

// float -> bf16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ u16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

union Frag {
    bf16x8 v;
    uint4 u;
};


// ------------------------------------------------------------ conv fwd ---
// Block: 256 threads = 4 waves; 64 consecutive output pixels of one row,
// wave w owns pixels 16w..16w+15 and every output channel tile.
// X [N][H][W][Cin], Wk [taps][CoutP][Cin] (CoutP = 16 * NT, zero padded),
// bias [CoutP] or null, Y [N][H][W][Cout] as bf16 or f32.
template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd(const u16 *__restrict__ X,
                                                  const u16 *__restrict__ Wk,
                                                  const float *__restrict__ bias,
                                                  void *__restrict__ Y, int H, int W, int Cin,
                                                  int Cout, int taps, int relu, int out_f32)
{
    const int n = blockIdx.z, r = blockIdx.y;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int c_base = blockIdx.x * 64 + wid * 16;
    const int CoutP = NT * 16;
    const int KT = taps * Cin;
    const int m = lane & 15, grp = lane >> 4;
    const int c = c_base + m;  // output pixel column of this lane's A row
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const size_t img = (size_t)n * H * W;
    for (int kc = 0; kc < KT; kc += 32) {
        const int k = kc + 8 * grp;
        Frag a;
        a.u = make_uint4(0, 0, 0, 0);
        int tap = 0, ci = 0;
        if (k < KT) {
            tap = k / Cin;
            ci = k - tap * Cin;
            int dr = taps == 9 ? tap / 3 - 1 : 0, dc = taps == 9 ? tap % 3 - 1 : 0;
            int rr = r + dr, cc = c + dc;
            if (rr >= 0 && rr < H && cc >= 0 && cc < W && c < W)
                a.u = *(const uint4 *)(X + ((img + (size_t)rr * W + cc) * Cin + ci));
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            Frag b;
            b.u = make_uint4(0, 0, 0, 0);
            if (k < KT) b.u = *(const uint4 *)(Wk + (((size_t)tap * CoutP + t * 16 + m) * Cin + ci));
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[t], 0, 0, 0);
        }
    }
    // D[pixel = 4*grp + i][co = 16t + m]
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + m;
        const float bb = (bias && co < Cout) ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int cc = c_base + 4 * grp + i;
            if (cc < W && co < Cout) {
                float v = acc[t][i] + bb;
                if (relu) v = fmaxf(v, 0.f);
                size_t o = (img + (size_t)r * W + cc) * Cout + co;
                if (out_f32) ((float *)Y)[o] = v;
                else ((u16 *)Y)[o] = f2bf(v);
            }
        }
    }
}

// ----------------------------------------------------------- conv wgrad ---
// Partial weight gradient of one tap over a chunk of 32*KCH pixels.
// dZ [P][Cout] (P = N*H*W pixels, Cout % 8 == 0), X [P][Cin] (Cin % 8 == 0),
// part [nchunk][taps][CoutP][CinP] f32, dbp [nchunk][CoutP] f32 (tap 0 pass).
// Block = 256 threads; LDS holds the chunk's dZ and shifted X transposed
// (channel-major, 32 pixels per row) so MFMA fragments are 16-byte reads.
constexpr int kWgPix = 32;
constexpr int kWgLd = 40;  // bf16 row stride (32 + 8 pad)
constexpr int kWgTiles = 32;  // 16x16 output tiles per wave: CoutP*CinP <= 128*256

__global__ __launch_bounds__(256) void k_conv_wgrad(const u16 *__restrict__ dZ,
                                                    const u16 *__restrict__ X,
                                                    float *__restrict__ part,
                                                    float *__restrict__ dbp, int N, int H, int W,
                                                    int Cin, int Cout, int taps, int kch)
{
    extern __shared__ u16 lds[];
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    u16 *sZ = lds;                         // [CoutP][kWgLd]
    u16 *sX = lds + (size_t)CoutP * kWgLd; // [CinP][kWgLd]
    const int chunk = blockIdx.x, tap = blockIdx.y;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = lane & 15, grp = lane >> 4;
    const int tilesM = CoutP / 16, tilesN = CinP / 16, ntiles = tilesM * tilesN;
    const size_t P = (size_t)N * H * W;
    const int dr = taps == 9 ? tap / 3 - 1 : 0, dc = taps == 9 ? tap % 3 - 1 : 0;
    // each wave owns tiles wid, wid+4, ... (at most kWgTiles per wave)
    f32x4 acc[kWgTiles];
#pragma unroll
    for (int i = 0; i < kWgTiles; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;  // per-thread bias-gradient partial (channel threadIdx.x)
    for (int kk = 0; kk < kch; ++kk) {
        const size_t p0 = ((size_t)chunk * kch + kk) * kWgPix;
        if (p0 >= P) break;
        __syncthreads();
        // stage: 32 pixels x channels, 8 channels per thread item
        const int zitems = kWgPix * (CoutP / 8), xitems = kWgPix * (CinP / 8);
        for (int it = threadIdx.x; it < zitems + xitems; it += 256) {
            const bool isz = it < zitems;
            const int j = isz ? it : it - zitems;
            const int C = isz ? Cout : Cin, CP = isz ? CoutP : CinP;
            const int px = j / (CP / 8), c8 = (j % (CP / 8)) * 8;
            const size_t p = p0 + px;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (p < P && c8 < C) {
                if (isz) {
                    v = *(const uint4 *)(dZ + p * Cout + c8);
                } else {
                    const int n = (int)(p / ((size_t)H * W));
                    const int rem = (int)(p - (size_t)n * H * W);
                    const int rr = rem / W + dr, cc = rem % W + dc;
                    if (rr >= 0 && rr < H && cc >= 0 && cc < W)
                        v = *(const uint4 *)(X + (((size_t)n * H + rr) * W + cc) * Cin + c8);
                }
            }
            u16 *dst = (isz ? sZ : sX) + (size_t)c8 * kWgLd + px;
            const u16 *e = (const u16 *)&v;
#pragma unroll
            for (int q = 0; q < 8; ++q) dst[(size_t)q * kWgLd] = e[q];
        }
        __syncthreads();
        if (tap == (taps == 9 ? 4 : 0) && (int)threadIdx.x < Cout)
            for (int px = 0; px < kWgPix; ++px) dbacc += bf2f(sZ[(size_t)threadIdx.x * kWgLd + px]);
#pragma unroll
        for (int i = 0; i < kWgTiles; ++i) {
            const int tt = wid + 4 * i;
            if (tt < ntiles) {
                const int tm = tt / tilesN, tn = tt % tilesN;
                Frag a, b;
                a.u = *(const uint4 *)(sZ + (size_t)(tm * 16 + m) * kWgLd + 8 * grp);
                b.u = *(const uint4 *)(sX + (size_t)(tn * 16 + m) * kWgLd + 8 * grp);
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[i], 0, 0, 0);
            }
        }
    }
    // D[co = 16 tm + 4 grp + i][ci = 16 tn + m], stored as [CoutP][Cin]
    float *dst = part + ((size_t)chunk * taps + tap) * CoutP * Cin;
#pragma unroll
    for (int i = 0; i < kWgTiles; ++i) {
        const int tt = wid + 4 * i;
        if (tt < ntiles) {
            const int tm = tt / tilesN, tn = tt % tilesN;
            const int ci = tn * 16 + m;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (ci < Cin) dst[(size_t)(tm * 16 + 4 * grp + q) * Cin + ci] = acc[i][q];
        }
    }
    if (tap == (taps == 9 ? 4 : 0) && (int)threadIdx.x < CoutP)
        dbp[(size_t)chunk * CoutP + threadIdx.x] = (int)threadIdx.x < Cout ? dbacc : 0.f;
}

// out[i] = sum_chunk part[chunk][i] in chunk order
__global__ __launch_bounds__(256) void k_sum_chunks(const float *__restrict__ part,
                                                    float *__restrict__ out, int nchunk,
                                                    size_t len)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int q = 0; q < nchunk; ++q) s += part[(size_t)q * len + i];
    out[i] = s;
}

// --------------------------------------------------------- elementwise ---
// dgrad weights: Wd[tap'][ci][co] = Wk[taps-1-tap'][co][ci], CinP rows padded.
__global__ void k_wflip(const u16 *__restrict__ Wk, u16 *__restrict__ Wd, int taps, int Cin,
                        int Cout, int CoutP, int CinP)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t total = (size_t)taps * CinP * Cout;
    if (i >= total) return;
    int co = (int)(i % Cout);
    size_t rest = i / Cout;
    int ci = (int)(rest % CinP);
    int tp = (int)(rest / CinP);
    u16 v = 0;
    if (ci < Cin) v = Wk[((size_t)(taps - 1 - tp) * CoutP + co) * Cin + ci];
    Wd[i] = v;
}

__global__ void k_relu_bwd(const u16 *__restrict__ dy, const u16 *__restrict__ y,
                           u16 *__restrict__ dz, size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    dz[i] = bf2f(y[i]) > 0.f ? dy[i] : (u16)0;
}

// 2x2 max pool, stride 2 (H, W even); idx records the winning sub-pixel.
__global__ void k_pool_fwd(const u16 *__restrict__ x, u16 *__restrict__ y,
                           uint8_t *__restrict__ idx, int N, int H, int W, int C)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    size_t total = (size_t)N * Ho * Wo * C;
    if (i >= total) return;
    int c = (int)(i % C);
    size_t p = i / C;
    int wo = (int)(p % Wo), ho = (int)((p / Wo) % Ho), n = (int)(p / ((size_t)Wo * Ho));
    float best = -INFINITY;
    int bi = 0;
    for (int q = 0; q < 4; ++q) {
        int hh = 2 * ho + q / 2, ww = 2 * wo + q % 2;
        float v = bf2f(x[(((size_t)n * H + hh) * W + ww) * C + c]);
        if (v > best) { best = v; bi = q; }
    }
    y[i] = f2bf(best);
    idx[i] = (uint8_t)bi;
}

__global__ void k_pool_bwd(const u16 *__restrict__ dy, const uint8_t *__restrict__ idx,
                           u16 *__restrict__ dx, int N, int H, int W, int C)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;  // over dx
    size_t total = (size_t)N * H * W * C;
    if (i >= total) return;
    int c = (int)(i % C);
    size_t p = i / C;
    int w = (int)(p % W), h = (int)((p / W) % H), n = (int)(p / ((size_t)W * H));
    const int Ho = H / 2, Wo = W / 2;
    size_t o = (((size_t)n * Ho + h / 2) * Wo + w / 2) * C + c;
    dx[i] = idx[o] == (uint8_t)((h % 2) * 2 + (w % 2)) ? dy[o] : (u16)0;
}

// depth-to-space: y[n][2i+a][2j+b][c] = t[n][i][j][(2a+b)*C + c]; mode 1 inverts.
__global__ void k_shuffle(const u16 *__restrict__ src, u16 *__restrict__ dst, int N, int Hin,
                          int Win, int C, int inverse)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;  // over the 2x image
    const int H = 2 * Hin, W = 2 * Win;
    size_t total = (size_t)N * H * W * C;
    if (i >= total) return;
    int c = (int)(i % C);
    size_t p = i / C;
    int w = (int)(p % W), h = (int)((p / W) % H), n = (int)(p / ((size_t)W * H));
    size_t t = (((size_t)n * Hin + h / 2) * Win + w / 2) * (4 * C) + ((h % 2) * 2 + (w % 2)) * C + c;
    if (!inverse) dst[i] = src[t];
    else dst[t] = src[i];
}

// channel concat: z[p][0:C1] = a[p], z[p][C1:C1+C2] = b[p]; inverse splits.
__global__ void k_concat(u16 *__restrict__ a, u16 *__restrict__ b, u16 *__restrict__ z, size_t P,
                         int C1, int C2, int inverse)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int C = C1 + C2;
    if (i >= P * C) return;
    size_t p = i / C;
    int c = (int)(i % C);
    u16 *s = c < C1 ? a + p * C1 + c : b + p * C2 + (c - C1);
    if (!inverse) z[i] = *s;
    else *s = z[i];
}

__global__ void k_add(const u16 *__restrict__ a, const u16 *__restrict__ b, u16 *__restrict__ z,
                      size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) z[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

__global__ void k_f32_to_bf16(const float *__restrict__ x, u16 *__restrict__ y, size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_bf16_to_f32(const u16 *__restrict__ x, float *__restrict__ y, size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = bf2f(x[i]);
}

// Adam on FP32 master weights; also refreshes the BF16 working copy.
__global__ void k_adam(float *__restrict__ w, float *__restrict__ mom, float *__restrict__ var,
                       const float *__restrict__ g, u16 *__restrict__ wb, size_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, float wd)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gi = g[i] + wd * w[i];
    float mi = b1 * mom[i] + (1.f - b1) * gi;
    float vi = b2 * var[i] + (1.f - b2) * gi * gi;
    mom[i] = mi;
    var[i] = vi;
    float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    float nw = w[i] - upd;
    w[i] = nw;
    if (wb) wb[i] = f2bf(nw);
}

// MSE over the first `used` of C channels of y (f32) against t (f32):
// per-block partial sums (f64) and the gradient dy = 2 (y - t) / count.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y,
                                             const float *__restrict__ t, float *__restrict__ dy,
                                             double *__restrict__ partial, size_t P, int C,
                                             int used, double inv_count)
{
    double acc = 0.0;
    for (int j = 0; j < 4; ++j) {
        size_t i = ((size_t)blockIdx.x * 4 + j) * 256 + threadIdx.x;
        if (i < P * C) {
            int c = (int)(i % C);
            float d = 0.f;
            if (c < used) {
                size_t p = i / C;
                d = y[i] - t[p * used + c];
                acc += (double)d * d;
            }
            if (dy) dy[i] = (float)(2.0 * inv_count) * d;
        }
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

inline unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

const char *dect_nn_last_error(void) { return g_nn_err; }

dect_status dect_nn_conv_fwd(const void *x, const void *w, const float *bias, void *y, int32_t N,
                             int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                             int32_t relu, int32_t out_f32, void *stream)
{
    if (!x || !w || !y || N <= 0 || H <= 0 || W <= 0 || Cin <= 0 || Cout <= 0)
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd: bad arguments");
    if (Cin % 8 != 0 || Cout > 256 || (ksize != 1 && ksize != 3))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd: Cin % 8, Cout <= 256, ksize in {1,3}");
    const int taps = ksize * ksize;
    const int NT = (Cout + 15) / 16;
    dim3 grid((W + 63) / 64, H, N);
    hipStream_t s = (hipStream_t)stream;
    const u16 *X = (const u16 *)x, *Wk = (const u16 *)w;
    switch (NT) {
#define CASE(nt) case nt: hipLaunchKernelGGL(k_conv_fwd<nt>, grid, dim3(256), 0, s, X, Wk, bias, y, H, W, Cin, Cout, taps, relu, out_f32); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

size_t dect_nn_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                               int32_t ksize)
{
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    const size_t P = (size_t)N * H * W;
    const int kch = 16;
    const size_t nchunk = (P + (size_t)kWgPix * kch - 1) / ((size_t)kWgPix * kch);
    (void)CinP;
    return nchunk * ((size_t)ksize * ksize * CoutP * Cin + CoutP) * sizeof(float);
}

dect_status dect_nn_conv_wgrad(const void *dz, const void *x, float *dw, float *db, int32_t N,
                               int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                               void *workspace, size_t ws_bytes, void *stream)
{
    if (!dz || !x || !dw || !db || !workspace || N <= 0 || H <= 0 || W <= 0)
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: bad arguments");
    if (Cin % 8 != 0 || Cout % 8 != 0 || Cin > 256 || Cout > 256 || (ksize != 1 && ksize != 3))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: Cin, Cout % 8 and <= 256");
    if (((Cout + 15) / 16) * ((Cin + 15) / 16) > 4 * kWgTiles)
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: Cout*Cin tile count too large");
    if (ws_bytes < dect_nn_wgrad_workspace(N, H, W, Cin, Cout, ksize))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: workspace too small");
    const int taps = ksize * ksize;
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    const size_t P = (size_t)N * H * W;
    const int kch = 16;
    const int nchunk = (int)((P + (size_t)kWgPix * kch - 1) / ((size_t)kWgPix * kch));
    float *part = (float *)workspace;
    float *dbp = part + (size_t)nchunk * taps * CoutP * Cin;
    hipStream_t s = (hipStream_t)stream;
    size_t lds = (size_t)(CoutP + CinP) * kWgLd * sizeof(u16);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(nchunk, taps), dim3(256), lds, s, (const u16 *)dz,
                       (const u16 *)x, part, dbp, N, H, W, Cin, Cout, taps, kch);
    NN_HIP(hipGetLastError());
    size_t len = (size_t)taps * CoutP * Cin;
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(len)), dim3(256), 0, s, part, dw, nchunk, len);
    NN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(CoutP)), dim3(256), 0, s, dbp, db, nchunk,
                       (size_t)CoutP);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_weight_flip(const void *w, void *wd, int32_t Cin, int32_t Cout, int32_t ksize,
                                void *stream)
{
    if (!w || !wd || Cin <= 0 || Cout <= 0) return nn_fail(DECT_ERR_INVALID_ARG, "weight_flip");
    const int taps = ksize * ksize;
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    size_t total = (size_t)taps * CinP * Cout;
    hipLaunchKernelGGL(k_wflip, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream,
                       (const u16 *)w, (u16 *)wd, taps, Cin, Cout, CoutP, CinP);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_relu_bwd(const void *dy, const void *y, void *dz, size_t n, void *stream)
{
    if (n == 0) return DECT_OK;
    hipLaunchKernelGGL(k_relu_bwd, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                       (const u16 *)dy, (const u16 *)y, (u16 *)dz, n);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_pool(const void *x, void *y, void *idx, int32_t N, int32_t H, int32_t W,
                         int32_t C, int32_t backward, void *stream)
{
    if (H % 2 || W % 2) return nn_fail(DECT_ERR_INVALID_ARG, "pool: H and W must be even");
    hipStream_t s = (hipStream_t)stream;
    if (!backward) {
        size_t total = (size_t)N * (H / 2) * (W / 2) * C;
        hipLaunchKernelGGL(k_pool_fwd, dim3(blocks(total)), dim3(256), 0, s, (const u16 *)x,
                           (u16 *)y, (uint8_t *)idx, N, H, W, C);
    } else {  // x = dy (pooled), y = dx (full)
        size_t total = (size_t)N * H * W * C;
        hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(total)), dim3(256), 0, s, (const u16 *)x,
                           (const uint8_t *)idx, (u16 *)y, N, H, W, C);
    }
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_shuffle(const void *src, void *dst, int32_t N, int32_t Hin, int32_t Win,
                            int32_t C, int32_t inverse, void *stream)
{
    size_t total = (size_t)N * 4 * Hin * Win * C;
    hipLaunchKernelGGL(k_shuffle, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream,
                       (const u16 *)src, (u16 *)dst, N, Hin, Win, C, inverse);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_concat(void *a, void *b, void *z, size_t P, int32_t C1, int32_t C2,
                           int32_t inverse, void *stream)
{
    size_t total = P * (size_t)(C1 + C2);
    hipLaunchKernelGGL(k_concat, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream,
                       (u16 *)a, (u16 *)b, (u16 *)z, P, C1, C2, inverse);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_add(const void *a, const void *b, void *z, size_t n, void *stream)
{
    if (n == 0) return DECT_OK;
    hipLaunchKernelGGL(k_add, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, (const u16 *)a,
                       (const u16 *)b, (u16 *)z, n);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_convert(const void *src, void *dst, size_t n, int32_t to_bf16, void *stream)
{
    if (n == 0) return DECT_OK;
    if (to_bf16)
        hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                           (const float *)src, (u16 *)dst, n);
    else
        hipLaunchKernelGGL(k_bf16_to_f32, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                           (const u16 *)src, (float *)dst, n);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_adam(float *w, float *m, float *v, const float *g, void *w_bf16, size_t n,
                         double lr, double beta1, double beta2, double eps, int32_t step,
                         double weight_decay, void *stream)
{
    if (n == 0) return DECT_OK;
    if (step < 1) return nn_fail(DECT_ERR_INVALID_ARG, "adam: step counts from 1");
    float c1 = (float)(1.0 - std::pow(beta1, step)), c2 = (float)(1.0 - std::pow(beta2, step));
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, w, m, v, g,
                       (u16 *)w_bf16, n, (float)lr, (float)beta1, (float)beta2, (float)eps, c1,
                       c2, (float)weight_decay);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

size_t dect_nn_mse_partials(size_t P, int32_t C) { return (P * C + 1023) / 1024; }

dect_status dect_nn_mse(const float *y, const float *t, float *dy, double *partial, size_t P,
                        int32_t C, int32_t used, void *stream)
{
    size_t nb = dect_nn_mse_partials(P, C);
    double inv = 1.0 / ((double)P * used);
    hipLaunchKernelGGL(k_mse, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, y, t, dy,
                       partial, P, C, used, inv);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

}  // extern "C"
