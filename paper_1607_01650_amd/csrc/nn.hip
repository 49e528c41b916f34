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

#include <algorithm>
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
// Block: 256 threads = 4 waves on a tile of TR x 32 output pixels of one
// image (TR = 2 MT).  Wave w owns the MT pixel tiles j = w MT .. w MT + MT - 1
// (tile j: row j / 2, columns 16 (j % 2) .. + 15) and every output-channel
// tile, so each weight fragment it loads feeds MT matrix-core steps.  The
// input window (TR + 2 rows x 34 columns with the halo for 3x3, TR x 32 for
// 1x1) is staged in LDS, at most 64 channels at a time, with 16-byte loads;
// the output tile goes back through LDS and leaves as 16-byte stores.
// X [N][H][W][Cin], Wk [taps][CoutP][Cin] (CoutP = 16 NT, zero padded),
// bias [CoutP] or null, Y [N][H][W][Cout] as bf16 or f32.
constexpr int kConvLds = 49152;  // bytes: max(window chunk, output tile)
constexpr int kConvChunk = 64;   // channels staged at a time

constexpr int conv_mt(int nt) { return nt <= 6 ? 4 : (nt <= 12 ? 2 : 1); }
static_assert(2 * conv_mt(6) * 32 * 96 * 2 <= kConvLds && 2 * conv_mt(12) * 32 * 192 * 2 <= kConvLds &&
                  2 * conv_mt(16) * 32 * 256 * 2 <= kConvLds,
              "a bf16 output tile must fit the LDS");
static_assert((2 * conv_mt(16) + 2) * 34 * (kConvChunk + 8) * 2 <= kConvLds &&
                  (2 * conv_mt(6) + 2) * 34 * (kConvChunk + 8) * 2 <= kConvLds,
              "the staged input window must fit the LDS");

template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd(const u16 *__restrict__ X,
                                                  const u16 *__restrict__ Wk,
                                                  const float *__restrict__ bias,
                                                  void *__restrict__ Y, int H, int W, int Cin,
                                                  int Cout, int ks, int relu, int out_f32)
{
    constexpr int MT = conv_mt(NT);
    constexpr int TR = 2 * MT;
    constexpr int CoutP = NT * 16;
    // dynamic LDS, sized by the launch to this layer's window and output
    // tile (conv_fwd_lds): small layers keep more blocks per CU
    extern __shared__ __align__(16) unsigned char lds_raw[];
    u16 *win = (u16 *)lds_raw;
    const int n = blockIdx.z, r0 = blockIdx.y * TR, c0 = blockIdx.x * 32;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = lane & 15, grp = lane >> 4;
    const int halo = ks == 3 ? 1 : 0;
    const int HR = TR + 2 * halo, HC = 32 + 2 * halo;
    const size_t img = (size_t)n * H * W;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int cc0 = 0; cc0 < Cin; cc0 += kConvChunk) {
        const int CC = min(kConvChunk, Cin - cc0);  // a multiple of 8
        const int PS = CC + 8;                       // LDS pixel stride (bf16)
        const int c8n = CC / 8;
        __syncthreads();
        for (int it = threadIdx.x; it < HR * HC * c8n; it += 256) {
            const int px = it / c8n, c8 = (it - px * c8n) * 8;
            const int hr = px / HC, hc = px - hr * HC;
            const int rr = r0 - halo + hr, cc = c0 - halo + hc;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (rr >= 0 && rr < H && cc >= 0 && cc < W)
                v = *(const uint4 *)(X + (img + (size_t)rr * W + cc) * Cin + cc0 + c8);
            *(uint4 *)(win + px * PS + c8) = v;
        }
        __syncthreads();
        if (CC % 32 == 0) {  // whole 32-channel K steps: no index division
            for (int tap = 0; tap < ks * ks; ++tap) {
                const int dr = ks == 3 ? tap / 3 : 0, dc = ks == 3 ? tap - 3 * (tap / 3) : 0;
                const u16 *wrow = Wk + ((size_t)tap * CoutP + m) * Cin + cc0 + 8 * grp;
                const u16 *arow = win + (dr * HC + dc) * PS + 8 * grp;
                for (int ci0 = 0; ci0 < CC; ci0 += 32) {
                    Frag b[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        b[t].u = *(const uint4 *)(wrow + (size_t)t * 16 * Cin + ci0);
#pragma unroll
                    for (int i = 0; i < MT; ++i) {
                        const int j = wid * MT + i;
                        const int orow = j >> 1, ocol = 16 * (j & 1) + m;
                        Frag a;
                        a.u = *(const uint4 *)(arow + (orow * HC + ocol) * PS + ci0);
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b[t].v,
                                                                                acc[i][t], 0, 0, 0);
                    }
                }
            }
            continue;
        }
        const int KT = ks * ks * CC;  // this chunk's K: (tap, channel), tap-major
        for (int kc = 0; kc < KT; kc += 32) {
            const int k = kc + 8 * grp;
            const bool kin = k < KT;
            const int tap = kin ? k / CC : 0;
            const int ci = kin ? k - tap * CC : 0;
            const int dr = ks == 3 ? tap / 3 : 0, dc = ks == 3 ? tap - 3 * (tap / 3) : 0;
            Frag b[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                b[t].u = make_uint4(0, 0, 0, 0);
                if (kin)
                    b[t].u = *(const uint4 *)(Wk + (((size_t)tap * CoutP + t * 16 + m) * Cin +
                                                    cc0 + ci));
            }
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int j = wid * MT + i;
                const int orow = j >> 1, ocol = 16 * (j & 1) + m;
                Frag a;
                a.u = make_uint4(0, 0, 0, 0);
                if (kin) a.u = *(const uint4 *)(win + ((orow + dr) * HC + ocol + dc) * PS + ci);
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b[t].v, acc[i][t], 0,
                                                                        0, 0);
            }
        }
    }
    // epilogue: D[pixel 4 grp + q of tile j][co = 16 t + m]
    if (out_f32 && (size_t)TR * 32 * CoutP * 4 > (size_t)kConvLds) {
        // an FP32 tile larger than the LDS: straight from the registers
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + m;
            const float bb = (bias && co < Cout) ? bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int j = wid * MT + i;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int rr = r0 + (j >> 1), cc = c0 + 16 * (j & 1) + 4 * grp + q;
                    if (rr < H && cc < W && co < Cout) {
                        float v = acc[i][t][q] + bb;
                        if (relu) v = fmaxf(v, 0.f);
                        ((float *)Y)[(img + (size_t)rr * W + cc) * Cout + co] = v;
                    }
                }
            }
        }
        return;
    }
    // otherwise through LDS [pixel][co] (at most kConvLds bytes: bf16 tiles
    // are TR * 32 * CoutP * 2 <= 49152 bytes for every NT)
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + m;
        const float bb = (bias && co < Cout) ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int j = wid * MT + i;
            const int pbase = (j >> 1) * 32 + 16 * (j & 1) + 4 * grp;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v = acc[i][t][q] + bb;
                if (relu) v = fmaxf(v, 0.f);
                const int p = pbase + q;
                if (out_f32) ((float *)lds_raw)[p * CoutP + co] = v;
                else ((u16 *)lds_raw)[p * CoutP + co] = f2bf(v);
            }
        }
    }
    __syncthreads();
    const int epv = out_f32 ? 4 : 8;  // elements per 16-byte store
    if (Cout % epv != 0) {            // channel counts off the 16-byte grid: one at a time
        for (int it = threadIdx.x; it < TR * 32 * Cout; it += 256) {
            const int p = it / Cout, e = it - p * Cout;
            const int rr = r0 + (p >> 5), cc = c0 + (p & 31);
            if (rr < H && cc < W) {
                const size_t o = (img + (size_t)rr * W + cc) * Cout + e;
                if (out_f32) ((float *)Y)[o] = ((const float *)lds_raw)[p * CoutP + e];
                else ((u16 *)Y)[o] = ((const u16 *)lds_raw)[p * CoutP + e];
            }
        }
        return;
    }
    const int vpp = Cout / epv;  // stores per pixel
    for (int it = threadIdx.x; it < TR * 32 * vpp; it += 256) {
        const int p = it / vpp, e = (it - p * vpp) * epv;
        const int rr = r0 + (p >> 5), cc = c0 + (p & 31);
        if (rr < H && cc < W) {
            const size_t o = (img + (size_t)rr * W + cc) * Cout + e;
            if (out_f32)
                *(uint4 *)((float *)Y + o) = *(const uint4 *)((const float *)lds_raw + p * CoutP + e);
            else
                *(uint4 *)((u16 *)Y + o) = *(const uint4 *)((const u16 *)lds_raw + p * CoutP + e);
        }
    }
}

// ----------------------------------------------------------- conv wgrad ---
// Partial weight gradient of one tap over a chunk of PIX * kch pixels.
// dZ [P][Cout] (P = N*H*W pixels, Cout % 8 == 0), X [P][Cin] (Cin % 8 == 0),
// part [nchunk][taps][CoutP][Cin] f32.  (The bias gradient is a separate
// column sum of dZ, k_bias_partial.)
// Block = 256 threads.  Each step stages PIX pixels of dZ and of the shifted
// X transposed in LDS (channel-major, pixel-contiguous rows), so the MFMA
// fragments (K = 32 pixels) are 16-byte reads, and every wave's TPW output
// tiles take PIX / 32 matrix-core steps per stage.  TPW is sized to the layer
// (tiles / 4 rounded up to 2, 4, 8, 16 or 24), which keeps the registers of
// small layers few and their blocks many per CU: other blocks' matrix work
// covers one block's staging loads.
constexpr size_t kWgLdsMax = 65536;

// 128 pixels per stage, or 64 when the staged channels (CoutP + CinP) would
// not fit 64 KB of LDS at 128.
inline int wgrad_pix(int CoutP, int CinP)
{
    return (size_t)(CoutP + CinP) * (128 + 8) * 2 <= kWgLdsMax ? 128 : 64;
}

template <int PIX, int TPW>
__global__ __launch_bounds__(256) void k_conv_wgrad(const u16 *__restrict__ dZ,
                                                    const u16 *__restrict__ X,
                                                    float *__restrict__ part, int N, int H, int W,
                                                    int Cin, int Cout, int taps, int kch)
{
    constexpr int LD = PIX + 8;  // bf16 row stride
    extern __shared__ u16 lds[];
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    u16 *sZ = lds;                       // [CoutP][LD]
    u16 *sX = lds + (size_t)CoutP * LD;  // [CinP][LD]
    const int chunk = blockIdx.x, tap = blockIdx.y;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = lane & 15, grp = lane >> 4;
    const int tilesN = CinP / 16, ntiles = (CoutP / 16) * tilesN;
    const size_t P = (size_t)N * H * W, HW = (size_t)H * W;
    const int dr = taps == 9 ? tap / 3 - 1 : 0, dc = taps == 9 ? tap % 3 - 1 : 0;
    // staging items: 4 consecutive pixels x 8 channels (four 16-byte loads,
    // transposed in registers into eight 8-byte LDS writes, one per channel)
    const int zitems = (PIX / 4) * (CoutP / 8), total = zitems + (PIX / 4) * (CinP / 8);
    // each wave owns tiles wid, wid + 4, ... (at most TPW per wave)
    f32x4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < kch; ++kk) {
        const size_t p0 = ((size_t)chunk * kch + kk) * PIX;
        if (p0 >= P) break;
        __syncthreads();  // the previous step's tiles are done with the LDS
        for (int it = threadIdx.x; it < total; it += 256) {
            const bool isz = it < zitems;
            const int j = isz ? it : it - zitems;
            const int C = isz ? Cout : Cin, CP8 = (isz ? CoutP : CinP) / 8;
            const int px4 = j / CP8, c8 = (j - px4 * CP8) * 8;
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = make_uint4(0, 0, 0, 0);
                const size_t p = p0 + 4 * px4 + u;
                if (p < P && c8 < C) {
                    if (isz) {
                        v[u] = *(const uint4 *)(dZ + p * Cout + c8);
                    } else {
                        const size_t n = p / HW;
                        const int rem = (int)(p - n * HW);
                        const int rr = rem / W + dr, cc = rem % W + dc;
                        if (rr >= 0 && rr < H && cc >= 0 && cc < W)
                            v[u] = *(const uint4 *)(X + ((n * H + rr) * W + cc) * Cin + c8);
                    }
                }
            }
            u16 *dst = (isz ? sZ : sX) + (size_t)c8 * LD + 4 * px4;
            const u16 *e0 = (const u16 *)&v[0], *e1 = (const u16 *)&v[1];
            const u16 *e2 = (const u16 *)&v[2], *e3 = (const u16 *)&v[3];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint2 w;
                w.x = (uint32_t)e0[q] | ((uint32_t)e1[q] << 16);
                w.y = (uint32_t)e2[q] | ((uint32_t)e3[q] << 16);
                *(uint2 *)(dst + (size_t)q * LD) = w;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int tt = wid + 4 * i;
            if (tt < ntiles) {
                const int tm = tt / tilesN, tn = tt - tm * tilesN;
#pragma unroll
                for (int ks = 0; ks < PIX; ks += 32) {
                    Frag a, b;
                    a.u = *(const uint4 *)(sZ + (size_t)(tm * 16 + m) * LD + ks + 8 * grp);
                    b.u = *(const uint4 *)(sX + (size_t)(tn * 16 + m) * LD + ks + 8 * grp);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[i], 0, 0, 0);
                }
            }
        }
    }
    // D[co = 16 tm + 4 grp + i][ci = 16 tn + m], stored as [CoutP][Cin]
    float *dst = part + ((size_t)chunk * taps + tap) * CoutP * Cin;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int tt = wid + 4 * i;
        if (tt < ntiles) {
            const int tm = tt / tilesN, tn = tt - tm * tilesN;
            const int ci = tn * 16 + m;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (ci < Cin) dst[(size_t)(tm * 16 + 4 * grp + q) * Cin + ci] = acc[i][q];
        }
    }
}

// Weight gradient of a 3x3 convolution, the three taps of one kernel row per
// block, for W a multiple of PIX: each step takes PIX pixels of one image
// row.  It stages dZ of those pixels (transposed, [co][pixel]) and the input
// row r + dr over columns c0-1 .. c0+PIX (transposed, [ci][column]) once, and
// each of the three taps dc reads its operand from that row at a column
// shift of 0, 1 or 2: 16-byte aligned for shift 0, rebuilt from an aligned
// 16-byte read and the next dword (funnel shift) for 1 and 2.  blockIdx.y =
// dr-row (0..2) x split; a block owns up to 4 TPW (tap, 16x16 output tile)
// pairs of its row.  part [nchunk][9][CoutP][Cin] f32, as k_conv_wgrad.
template <int PIX, int TPW>
__global__ __launch_bounds__(256) void k_conv_wgrad_rows(const u16 *__restrict__ dZ,
                                                         const u16 *__restrict__ X,
                                                         float *__restrict__ part, int N, int H,
                                                         int W, int Cin, int Cout, int kch,
                                                         int nsplit)
{
    constexpr int LD = PIX + 8;  // bf16 row stride of both staged arrays
    extern __shared__ u16 lds[];
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    u16 *sZ = lds;                       // [CoutP][LD]
    u16 *sX = lds + (size_t)CoutP * LD;  // [CinP][LD]: element k is column c0 - 1 + k
    const int chunk = blockIdx.x, d = blockIdx.y / nsplit, split = blockIdx.y - d * nsplit;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = lane & 15, grp = lane >> 4;
    const int tilesN = CinP / 16, ntiles = (CoutP / 16) * tilesN, npairs = 3 * ntiles;
    const int pair0 = split * 4 * TPW;
    const size_t P = (size_t)N * H * W, HW = (size_t)H * W;
    const int K4 = (PIX + 4) / 4;  // 4-column groups of the staged row (columns up to c0 + PIX + 2)
    const int zitems = (PIX / 4) * (CoutP / 8), xitems = K4 * (CinP / 8);
    f32x4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < kch; ++kk) {
        const size_t p0 = ((size_t)chunk * kch + kk) * PIX;
        if (p0 >= P) break;
        const size_t n = p0 / HW;
        const int rem = (int)(p0 - n * HW);
        const int r = rem / W, c0 = rem - r * W;
        const int rr = r + d - 1;
        __syncthreads();  // the previous step's tiles are done with the LDS
        for (int it = threadIdx.x; it < zitems + xitems; it += 256) {
            uint4 v[4];
            u16 *dst;
            if (it < zitems) {
                const int CP8 = CoutP / 8;
                const int px4 = it / CP8, c8 = (it - px4 * CP8) * 8;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    v[u] = make_uint4(0, 0, 0, 0);
                    if (c8 < Cout) v[u] = *(const uint4 *)(dZ + (p0 + 4 * px4 + u) * Cout + c8);
                }
                dst = sZ + (size_t)c8 * LD + 4 * px4;
            } else {
                const int j = it - zitems, CP8 = CinP / 8;
                const int k4 = j / CP8, c8 = (j - k4 * CP8) * 8;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    v[u] = make_uint4(0, 0, 0, 0);
                    const int cc = c0 - 1 + 4 * k4 + u;
                    if (c8 < Cin && rr >= 0 && rr < H && cc >= 0 && cc < W)
                        v[u] = *(const uint4 *)(X + ((n * H + rr) * W + cc) * Cin + c8);
                }
                dst = sX + (size_t)c8 * LD + 4 * k4;
            }
            const u16 *e0 = (const u16 *)&v[0], *e1 = (const u16 *)&v[1];
            const u16 *e2 = (const u16 *)&v[2], *e3 = (const u16 *)&v[3];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint2 w;
                w.x = (uint32_t)e0[q] | ((uint32_t)e1[q] << 16);
                w.y = (uint32_t)e2[q] | ((uint32_t)e3[q] << 16);
                *(uint2 *)(dst + (size_t)q * LD) = w;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int pi = pair0 + wid + 4 * i;
            if (pi < npairs) {
                const int sh = pi / ntiles, tt = pi - sh * ntiles;  // column shift 0..2
                const int tm = tt / tilesN, tn = tt - tm * tilesN;
                const u16 *zr = sZ + (size_t)(tm * 16 + m) * LD + 8 * grp;
                const u16 *xr = sX + (size_t)(tn * 16 + m) * LD + 8 * grp;
#pragma unroll
                for (int ks = 0; ks < PIX; ks += 32) {
                    Frag a, b;
                    a.u = *(const uint4 *)(zr + ks);
                    const uint4 v = *(const uint4 *)(xr + ks);
                    if (sh == 0) {
                        b.u = v;
                    } else {
                        const uint32_t nx = *(const uint32_t *)(xr + ks + 8);
                        if (sh == 2) {
                            b.u = make_uint4(v.y, v.z, v.w, nx);
                        } else {
                            b.u = make_uint4(__builtin_amdgcn_alignbit(v.y, v.x, 16),
                                             __builtin_amdgcn_alignbit(v.z, v.y, 16),
                                             __builtin_amdgcn_alignbit(v.w, v.z, 16),
                                             __builtin_amdgcn_alignbit(nx, v.w, 16));
                        }
                    }
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[i], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int pi = pair0 + wid + 4 * i;
        if (pi < npairs) {
            const int sh = pi / ntiles, tt = pi - sh * ntiles;
            const int tm = tt / tilesN, tn = tt - tm * tilesN;
            float *dst = part + ((size_t)chunk * 9 + 3 * d + sh) * CoutP * Cin;
            const int ci = tn * 16 + m;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (ci < Cin) dst[(size_t)(tm * 16 + 4 * grp + q) * Cin + ci] = acc[i][q];
        }
    }
}

// Bias gradient partials: dbp[b][co] = sum of dZ[p][co] over the pixels of
// block b (kBiasPix of them).  Thread t sums channel group t % (Cout / 8) over
// pixels t / (Cout / 8), + 256 / (Cout / 8), ...; the threads of a group are
// then added in thread order.
constexpr int kBiasPix = 2048;
__global__ __launch_bounds__(256) void k_bias_partial(const u16 *__restrict__ dZ,
                                                      float *__restrict__ dbp, size_t P, int Cout,
                                                      int CoutP)
{
    __shared__ float red[256][9];
    const int g8 = Cout / 8;  // Cout % 8 == 0, Cout <= 256 -> g8 <= 32
    const int grpi = threadIdx.x % g8, row = threadIdx.x / g8, rows = 256 / g8;
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const size_t p0 = (size_t)blockIdx.x * kBiasPix;
    if (row < rows)
        for (int px = row; px < kBiasPix; px += rows) {
            const size_t p = p0 + px;
            if (p >= P) break;
            const uint4 v = *(const uint4 *)(dZ + p * Cout + 8 * grpi);
            const u16 *e = (const u16 *)&v;
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] += bf2f(e[q]);
        }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[threadIdx.x][q] = a[q];
    __syncthreads();
    if ((int)threadIdx.x < CoutP) {
        const int co = threadIdx.x;
        float sum = 0.f;
        if (co < Cout)
            for (int r = 0; r < rows; ++r) sum += red[r * g8 + co / 8][co % 8];
        dbp[(size_t)blockIdx.x * CoutP + co] = sum;
    }
}

// seg[s][i] = sum over chunks q in [s L, min(nchunk, (s + 1) L)) of
// part[q][i]; four interleaved running sums, combined in a fixed order.
__global__ __launch_bounds__(256) void k_sum_seg(const float *__restrict__ part,
                                                 float *__restrict__ seg, int nchunk, size_t len,
                                                 int L)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const int q0 = blockIdx.y * L, q1 = min(nchunk, q0 + L);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int q = q0;
    for (; q + 4 <= q1; q += 4) {
        a0 += part[(size_t)q * len + i];
        a1 += part[(size_t)(q + 1) * len + i];
        a2 += part[(size_t)(q + 2) * len + i];
        a3 += part[(size_t)(q + 3) * len + i];
    }
    for (; q < q1; ++q) a0 += part[(size_t)q * len + i];
    seg[(size_t)blockIdx.y * len + i] = (a0 + a1) + (a2 + a3);
}

// out[i] = sum_s seg[s][i] in segment order
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

// Segments for summing nchunk partials of len values: enough blocks to
// spread the reads over the GPU, at least 8 chunks per segment.
inline int sum_segments(int nchunk, size_t len)
{
    const size_t bx = (len + 255) / 256;
    size_t S = (2048 + bx - 1) / bx;
    S = std::min<size_t>(S, (size_t)std::max(1, nchunk / 8));
    return (int)std::max<size_t>(1, S);
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

// the same, 8 elements (16 bytes) per thread; n8 = n / 8
__global__ void k_relu_bwd8(const uint4 *__restrict__ dy, const uint4 *__restrict__ y,
                            uint4 *__restrict__ dz, size_t n8)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n8) return;
    uint4 a = dy[i], b = y[i], r;
    const u16 *ea = (const u16 *)&a, *eb = (const u16 *)&b;
    u16 *er = (u16 *)&r;
#pragma unroll
    for (int q = 0; q < 8; ++q) er[q] = bf2f(eb[q]) > 0.f ? ea[q] : (u16)0;
    dz[i] = r;
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

__global__ void k_add8(const uint4 *__restrict__ a, const uint4 *__restrict__ b,
                       uint4 *__restrict__ z, size_t n8)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n8) return;
    uint4 x = a[i], y = b[i], r;
    const u16 *ex = (const u16 *)&x, *ey = (const u16 *)&y;
    u16 *er = (u16 *)&r;
#pragma unroll
    for (int q = 0; q < 8; ++q) er[q] = f2bf(bf2f(ex[q]) + bf2f(ey[q]));
    z[i] = r;
}

// channel concat / split in 8-channel (16-byte) pieces (C1, C2 % 8 == 0)
__global__ void k_concat8(uint4 *__restrict__ a, uint4 *__restrict__ b, uint4 *__restrict__ z,
                          size_t P, int C1, int C2, int inverse)
{
    const int g1 = C1 / 8, g = (C1 + C2) / 8;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= P * g) return;
    size_t p = i / g;
    int c = (int)(i - p * g);
    uint4 *s = c < g1 ? a + p * g1 + c : b + p * (g - g1) + (c - g1);
    if (!inverse) z[i] = *s;
    else *s = z[i];
}

// depth-to-space in 8-channel pieces (C % 8 == 0)
__global__ void k_shuffle8(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int N, int Hin,
                           int Win, int C, int inverse)
{
    const int g = C / 8;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;  // over the 2x image, 8 channels each
    const int H = 2 * Hin, W = 2 * Win;
    size_t total = (size_t)N * H * W * g;
    if (i >= total) return;
    int c = (int)(i % g);
    size_t p = i / g;
    int w = (int)(p % W), h = (int)((p / W) % H), n = (int)(p / ((size_t)W * H));
    size_t t = (((size_t)n * Hin + h / 2) * Win + w / 2) * (4 * g) + ((h % 2) * 2 + (w % 2)) * g + c;
    if (!inverse) dst[i] = src[t];
    else dst[t] = src[i];
}

// 2x2 max pool, 8 channels per thread (C % 8 == 0)
__global__ void k_pool_fwd8(const u16 *__restrict__ x, u16 *__restrict__ y,
                            uint8_t *__restrict__ idx, int N, int H, int W, int C)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2, g = C / 8;
    size_t total = (size_t)N * Ho * Wo * g;
    if (i >= total) return;
    int c = (int)(i % g) * 8;
    size_t p = i / g;
    int wo = (int)(p % Wo), ho = (int)((p / Wo) % Ho), n = (int)(p / ((size_t)Wo * Ho));
    float best[8];
    uint8_t bi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) { best[q] = -INFINITY; bi[q] = 0; }
    for (int s = 0; s < 4; ++s) {
        int hh = 2 * ho + s / 2, ww = 2 * wo + s % 2;
        uint4 v = *(const uint4 *)(x + (((size_t)n * H + hh) * W + ww) * C + c);
        const u16 *e = (const u16 *)&v;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float f = bf2f(e[q]);
            if (f > best[q]) { best[q] = f; bi[q] = (uint8_t)s; }
        }
    }
    uint4 r;
    u16 *er = (u16 *)&r;
    uint2 ri;
    uint8_t *eri = (uint8_t *)&ri;
#pragma unroll
    for (int q = 0; q < 8; ++q) { er[q] = f2bf(best[q]); eri[q] = bi[q]; }
    const size_t o = p * C + c;
    *(uint4 *)(y + o) = r;
    *(uint2 *)(idx + o) = ri;
}

__global__ void k_pool_bwd8(const u16 *__restrict__ dy, const uint8_t *__restrict__ idx,
                            u16 *__restrict__ dx, int N, int H, int W, int C)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;  // over dx, 8 channels each
    const int g = C / 8;
    size_t total = (size_t)N * H * W * g;
    if (i >= total) return;
    int c = (int)(i % g) * 8;
    size_t p = i / g;
    int w = (int)(p % W), h = (int)((p / W) % H), n = (int)(p / ((size_t)W * H));
    const int Ho = H / 2, Wo = W / 2;
    size_t o = (((size_t)n * Ho + h / 2) * Wo + w / 2) * C + c;
    const uint4 d = *(const uint4 *)(dy + o);
    const uint2 ix = *(const uint2 *)(idx + o);
    const u16 *ed = (const u16 *)&d;
    const uint8_t *ei = (const uint8_t *)&ix;
    const uint8_t me = (uint8_t)((h % 2) * 2 + (w % 2));
    uint4 r;
    u16 *er = (u16 *)&r;
#pragma unroll
    for (int q = 0; q < 8; ++q) er[q] = ei[q] == me ? ed[q] : (u16)0;
    *(uint4 *)(dx + p * C + c) = r;
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

// LDS bytes k_conv_fwd<NT> uses for a layer: the largest staged input window
// and, unless an FP32 tile goes straight from the registers, the output tile.
static size_t conv_fwd_lds(int nt, int Cin, int ks, int out_f32)
{
    const int mt = conv_mt(nt), tr = 2 * mt, halo = ks == 3 ? 1 : 0;
    const size_t cc = (size_t)std::min(kConvChunk, Cin);
    const size_t win = (size_t)(tr + 2 * halo) * (32 + 2 * halo) * (cc + 8) * 2;
    const size_t tile = (size_t)tr * 32 * nt * 16 * (out_f32 ? 4 : 2);
    const bool tile_in_lds = !(out_f32 && tile > (size_t)kConvLds);
    return std::max(win, tile_in_lds ? tile : (size_t)0);
}

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
    const int NT = (Cout + 15) / 16;
    hipStream_t s = (hipStream_t)stream;
    const u16 *X = (const u16 *)x, *Wk = (const u16 *)w;
    switch (NT) {
#define CASE(nt)                                                                         \
    case nt: {                                                                           \
        dim3 grid((W + 31) / 32, (H + 2 * conv_mt(nt) - 1) / (2 * conv_mt(nt)), N);      \
        hipLaunchKernelGGL(k_conv_fwd<nt>, grid, dim3(256),                                \
                           (unsigned)conv_fwd_lds(nt, Cin, ksize, out_f32), s, X, Wk, bias, y, \
                           H, W, Cin, Cout, ksize, relu, out_f32);                       \
    } break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

// Pixel steps per wgrad block: enough blocks (chunks x taps) to fill the
// GPU several times over, at most 4096 pixels per block.
static int wgrad_steps(size_t P, int taps, int pix)
{
    const size_t steps = (P + pix - 1) / pix;
    const size_t want_chunks = (4096 + (size_t)taps - 1) / taps;
    size_t kch = (steps + want_chunks - 1) / want_chunks;
    return (int)std::max<size_t>(1, std::min<size_t>(4096 / pix, kch));
}

struct WgradPlan {
    int rows;                 // 1: k_conv_wgrad_rows (all taps per block), 0: per tap
    int pix, kch, nchunk, nsplit, tpw, nbias, segw, segb;
    size_t lds, part_floats, dbp_floats, segw_floats, segb_floats;
};

static WgradPlan wgrad_plan(int N, int H, int W, int Cin, int Cout, int ksize)
{
    WgradPlan q;
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    const size_t P = (size_t)N * H * W;
    const int taps = ksize * ksize;
    const int ntiles = (CoutP / 16) * (CinP / 16);
    q.rows = 0;
    q.nsplit = 1;
    if (ksize == 3) {  // the row-window kernel: widest pixel step that fits
        for (int pix : {128, 64, 32}) {
            const size_t lds = (size_t)(CoutP + CinP) * (pix + 8) * 2;
            if (W % pix == 0 && lds <= kWgLdsMax) {
                q.rows = 1;
                q.pix = pix;
                q.lds = lds;
                break;
            }
        }
    }
    if (q.rows) {
        const int pairs = 3 * ntiles;  // per kernel row
        q.tpw = pairs <= 16 ? 4 : (pairs <= 32 ? 8 : 16);
        q.nsplit = (pairs + 4 * q.tpw - 1) / (4 * q.tpw);
        const size_t steps = P / q.pix;
        const size_t want = (2048 + 3 * (size_t)q.nsplit - 1) / (3 * q.nsplit);  // chunks
        q.kch = (int)std::max<size_t>(1, std::min<size_t>(4096 / q.pix, (steps + want - 1) / want));
    } else {
        q.pix = wgrad_pix(CoutP, CinP);
        q.lds = (size_t)(CoutP + CinP) * (q.pix + 8) * 2;
        q.tpw = (ntiles + 3) / 4;
        q.kch = wgrad_steps(P, taps, q.pix);
    }
    q.nchunk = (int)((P + (size_t)q.pix * q.kch - 1) / ((size_t)q.pix * q.kch));
    const size_t len = (size_t)taps * CoutP * Cin;
    q.nbias = (int)((P + kBiasPix - 1) / kBiasPix);
    q.segw = sum_segments(q.nchunk, len);
    q.segb = sum_segments(q.nbias, (size_t)CoutP);
    q.part_floats = (size_t)q.nchunk * len;
    q.dbp_floats = (size_t)q.nbias * CoutP;
    q.segw_floats = (size_t)q.segw * len;
    q.segb_floats = (size_t)q.segb * CoutP;
    return q;
}

size_t dect_nn_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                               int32_t ksize)
{
    const WgradPlan q = wgrad_plan(N, H, W, Cin, Cout, ksize);
    return (q.part_floats + q.dbp_floats + q.segw_floats + q.segb_floats) * sizeof(float);
}

dect_status dect_nn_conv_wgrad(const void *dz, const void *x, float *dw, float *db, int32_t N,
                               int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                               void *workspace, size_t ws_bytes, void *stream)
{
    if (!dz || !x || !dw || !db || !workspace || N <= 0 || H <= 0 || W <= 0)
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: bad arguments");
    if (Cin % 8 != 0 || Cout % 8 != 0 || Cin > 256 || Cout > 256 || (ksize != 1 && ksize != 3))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: Cin, Cout % 8 and <= 256");
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    const int ntiles = (CoutP / 16) * (CinP / 16);
    if (ntiles > 4 * 24) return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: Cout*Cin tile count too large");
    if (ws_bytes < dect_nn_wgrad_workspace(N, H, W, Cin, Cout, ksize))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: workspace too small");
    const int taps = ksize * ksize;
    const WgradPlan q = wgrad_plan(N, H, W, Cin, Cout, ksize);
    float *part = (float *)workspace;
    float *dbp = part + q.part_floats;
    float *segw = dbp + q.dbp_floats;
    float *segb = segw + q.segw_floats;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = q.lds;
    if (lds > kWgLdsMax) return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: too many channels");
    const int tpw = q.tpw;
    const dim3 grid(q.nchunk, taps);
    const u16 *Z = (const u16 *)dz, *Xp = (const u16 *)x;
#define WR(pix, t)                                                                         \
    hipLaunchKernelGGL((k_conv_wgrad_rows<pix, t>), dim3(q.nchunk, 3 * q.nsplit), dim3(256), \
                       lds, s, Z, Xp, part, N, H, W, Cin, Cout, q.kch, q.nsplit)
#define WG(pix, t)                                                                          \
    hipLaunchKernelGGL((k_conv_wgrad<pix, t>), grid, dim3(256), lds, s, Z, Xp, part, N, H, W,  \
                       Cin, Cout, taps, q.kch)
#define WRT(pix)                           \
    if (tpw == 4) WR(pix, 4);              \
    else if (tpw == 8) WR(pix, 8);         \
    else WR(pix, 16);
    if (q.rows) {
        if (q.pix == 128) { WRT(128) }
        else if (q.pix == 64) { WRT(64) }
        else { WRT(32) }
    } else if (q.pix == 128) {
        if (tpw <= 2) WG(128, 2);
        else if (tpw <= 4) WG(128, 4);
        else if (tpw <= 8) WG(128, 8);
        else if (tpw <= 16) WG(128, 16);
        else WG(128, 24);
    } else {
        if (tpw <= 2) WG(64, 2);
        else if (tpw <= 4) WG(64, 4);
        else if (tpw <= 8) WG(64, 8);
        else if (tpw <= 16) WG(64, 16);
        else WG(64, 24);
    }
#undef WG
#undef WR
#undef WRT
    NN_HIP(hipGetLastError());
    const size_t len = (size_t)taps * CoutP * Cin;
    const int Lw = (q.nchunk + q.segw - 1) / q.segw, Lb = (q.nbias + q.segb - 1) / q.segb;
    hipLaunchKernelGGL(k_sum_seg, dim3(blocks(len), q.segw), dim3(256), 0, s, part, segw,
                       q.nchunk, len, Lw);
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(len)), dim3(256), 0, s, segw, dw, q.segw, len);
    hipLaunchKernelGGL(k_bias_partial, dim3(q.nbias), dim3(256), 0, s, Z, dbp, (size_t)N * H * W,
                       Cout, CoutP);
    hipLaunchKernelGGL(k_sum_seg, dim3(blocks(CoutP), q.segb), dim3(256), 0, s, dbp, segb,
                       q.nbias, (size_t)CoutP, Lb);
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(CoutP)), dim3(256), 0, s, segb, db, q.segb,
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

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

dect_status dect_nn_relu_bwd(const void *dy, const void *y, void *dz, size_t n, void *stream)
{
    if (n == 0) return DECT_OK;
    if (n % 8 == 0 && aligned16(dy) && aligned16(y) && aligned16(dz))
        hipLaunchKernelGGL(k_relu_bwd8, dim3(blocks(n / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint4 *)dy, (const uint4 *)y, (uint4 *)dz, n / 8);
    else
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
    const bool v8 = C % 8 == 0 && aligned16(x) && aligned16(y) && ((uintptr_t)idx & 7) == 0;
    if (!backward) {
        size_t total = (size_t)N * (H / 2) * (W / 2) * C;
        if (v8)
            hipLaunchKernelGGL(k_pool_fwd8, dim3(blocks(total / 8)), dim3(256), 0, s,
                               (const u16 *)x, (u16 *)y, (uint8_t *)idx, N, H, W, C);
        else
            hipLaunchKernelGGL(k_pool_fwd, dim3(blocks(total)), dim3(256), 0, s, (const u16 *)x,
                               (u16 *)y, (uint8_t *)idx, N, H, W, C);
    } else {  // x = dy (pooled), y = dx (full)
        size_t total = (size_t)N * H * W * C;
        if (v8)
            hipLaunchKernelGGL(k_pool_bwd8, dim3(blocks(total / 8)), dim3(256), 0, s,
                               (const u16 *)x, (const uint8_t *)idx, (u16 *)y, N, H, W, C);
        else
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
    if (C % 8 == 0 && aligned16(src) && aligned16(dst))
        hipLaunchKernelGGL(k_shuffle8, dim3(blocks(total / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint4 *)src, (uint4 *)dst, N, Hin, Win, C, inverse);
    else
        hipLaunchKernelGGL(k_shuffle, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream,
                           (const u16 *)src, (u16 *)dst, N, Hin, Win, C, inverse);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_concat(void *a, void *b, void *z, size_t P, int32_t C1, int32_t C2,
                           int32_t inverse, void *stream)
{
    size_t total = P * (size_t)(C1 + C2);
    if (C1 % 8 == 0 && C2 % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(z))
        hipLaunchKernelGGL(k_concat8, dim3(blocks(total / 8)), dim3(256), 0, (hipStream_t)stream,
                           (uint4 *)a, (uint4 *)b, (uint4 *)z, P, C1, C2, inverse);
    else
        hipLaunchKernelGGL(k_concat, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream,
                           (u16 *)a, (u16 *)b, (u16 *)z, P, C1, C2, inverse);
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_add(const void *a, const void *b, void *z, size_t n, void *stream)
{
    if (n == 0) return DECT_OK;
    if (n % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(z))
        hipLaunchKernelGGL(k_add8, dim3(blocks(n / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint4 *)a, (const uint4 *)b, (uint4 *)z, n / 8);
    else
        hipLaunchKernelGGL(k_add, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                           (const u16 *)a, (const u16 *)b, (u16 *)z, n);
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
