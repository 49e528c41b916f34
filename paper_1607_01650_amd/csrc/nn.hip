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
#include <array>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>

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

// The output tile [TR * 32 pixels][CoutP] staged in LDS (bf16, or FP32 with
// out_f32) to Y [.][H][W][Cout] as 16-byte stores where the channel count
// allows, zero where mask (when given) is not positive.
template <int CoutP>
__device__ __forceinline__ void conv_store_tile(const unsigned char *lds_raw, void *__restrict__ Y,
                                                const u16 *__restrict__ mask, size_t img, int r0,
                                                int c0, int TR, int H, int W, int Cout,
                                                int out_f32)
{
    const int epv = out_f32 ? 4 : 8;  // elements per 16-byte store
    if (Cout % epv != 0) {            // channel counts off the 16-byte grid: one at a time
        for (int it = threadIdx.x; it < TR * 32 * Cout; it += 256) {
            const int p = it / Cout, e = it - p * Cout;
            const int rr = r0 + (p >> 5), cc = c0 + (p & 31);
            if (rr < H && cc < W) {
                const size_t o = (img + (size_t)rr * W + cc) * Cout + e;
                const bool keep = !mask || bf2f(mask[o]) > 0.f;
                if (out_f32) ((float *)Y)[o] = keep ? ((const float *)lds_raw)[p * CoutP + e] : 0.f;
                else ((u16 *)Y)[o] = keep ? ((const u16 *)lds_raw)[p * CoutP + e] : (u16)0;
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
            if (out_f32) {
                uint4 v = *(const uint4 *)((const float *)lds_raw + p * CoutP + e);
                if (mask) {
                    const uint2 mk = *(const uint2 *)(mask + o);
                    const u16 *em = (const u16 *)&mk;
                    uint32_t *ev = (uint32_t *)&v;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (!(bf2f(em[q]) > 0.f)) ev[q] = 0u;
                }
                *(uint4 *)((float *)Y + o) = v;
            } else {
                uint4 v = *(const uint4 *)((const u16 *)lds_raw + p * CoutP + e);
                if (mask) {
                    const uint4 mk = *(const uint4 *)(mask + o);
                    const u16 *em = (const u16 *)&mk;
                    u16 *ev = (u16 *)&v;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (!(bf2f(em[q]) > 0.f)) ev[q] = 0;
                }
                *(uint4 *)((u16 *)Y + o) = v;
            }
        }
    }
}

template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd(const u16 *__restrict__ X,
                                                  const u16 *__restrict__ Wk,
                                                  const float *__restrict__ bias,
                                                  void *__restrict__ Y, int H, int W, int Cin,
                                                  int Cout, int ks, int relu, int out_f32,
                                                  const u16 *__restrict__ mask)
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
                        const size_t o = (img + (size_t)rr * W + cc) * Cout + co;
                        float v = acc[i][t][q] + bb;
                        if (relu) v = fmaxf(v, 0.f);
                        if (mask && !(bf2f(mask[o]) > 0.f)) v = 0.f;
                        ((float *)Y)[o] = v;
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
    conv_store_tile<CoutP>(lds_raw, Y, mask, img, r0, c0, TR, H, W, Cout, out_f32);
}

// ------------------------------------------------------ conv fwd, 3x3 ---
// The 3x3 forward / input-gradient convolution for Cout <= 128 and Cin >= 16.  Block: 4
// waves on TR x 32 output pixels of one image (TR = 2 MT); wave w takes the
// column half w & 1 and the MT rows (w >> 1) MT .. of the tile.  Input
// channels go in chunks of 32 (zero beyond Cin): per chunk the block stages
// the input window (TR + 2 rows x 34 columns) and the chunk's weights of all
// nine taps in LDS, each with 16-byte loads issued in groups of eight before
// their LDS writes.  Then for each column shift dc a wave reads the MT + 2
// window-row fragments it needs once and uses each for the three kernel rows
// dr (output row i takes window row i + dr), so a window fragment feeds up
// to 3 NT matrix-core steps and a weight fragment MT.  Pixel and weight rows
// are 80 bytes apart in LDS: a 16-lane fragment read touches every bank once.
constexpr int kC3Chunk = 32;
constexpr int kC3PS = kC3Chunk + 8;  // bf16 stride of a staged pixel or weight row
constexpr int conv3_mt(int) { return 4; }
// the 3x3 kernel up to 128 output channels from at least 16 input channels
// (its 32-channel chunks waste the matrix cores on fewer); its LDS (the
// weights of 128 output channels take 92 KB) fits the 160 KB of a CU
inline bool conv3_use(int nt, int cin) { return cin >= 16 && nt <= 8; }
constexpr size_t kC3LdsMax = 163840;

__host__ __device__ constexpr size_t conv3_lds(int nt, int out_f32)
{
    const size_t tr = 2 * conv3_mt(nt);
    const size_t stage = ((tr + 2) * 34 + 9 * 16 * (size_t)nt) * kC3PS * 2;
    const size_t tile = tr * 32 * 16 * (size_t)nt * (out_f32 ? 4 : 2);
    return stage > tile ? stage : tile;
}
static_assert(conv3_lds(8, 1) <= kC3LdsMax, "the 3x3 kernel's LDS must fit a CU");

// n items of 16 bytes: item k of this thread is it = threadIdx.x + 256 k;
// src(it) gives the global address (or null: zero), dst(it) the LDS one.
// Loads go out in groups of eight before their writes.
template <int NIT, class Src, class Dst>
__device__ __forceinline__ void stage16(int n, Src src, Dst dst)
{
#pragma unroll
    for (int g = 0; g < NIT; g += 8) {
        uint4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int it = threadIdx.x + 256 * (g + k);
            v[k] = make_uint4(0, 0, 0, 0);
            if (g + k < NIT && it < n) {
                const u16 *p = src(it);
                if (p) v[k] = *(const uint4 *)p;
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int it = threadIdx.x + 256 * (g + k);
            if (g + k < NIT && it < n) *(uint4 *)dst(it) = v[k];
        }
    }
}

template <int NT>
__global__ __launch_bounds__(256) void k_conv3(const u16 *__restrict__ X,
                                               const u16 *__restrict__ Wk,
                                               const float *__restrict__ bias,
                                               void *__restrict__ Y, int H, int W, int Cin,
                                               int Cout, int relu, int out_f32,
                                               const u16 *__restrict__ mask)
{
    constexpr int MT = conv3_mt(NT), TR = 2 * MT, CoutP = 16 * NT;
    constexpr int HR = TR + 2, HC = 34;
    constexpr int NWIN = HR * HC * 4, NWTS = 9 * CoutP * 4;  // 16-byte items
    extern __shared__ __align__(16) unsigned char lds_raw[];
    u16 *win = (u16 *)lds_raw;            // [HR][HC][kC3PS]
    u16 *wts = win + HR * HC * kC3PS;     // [9][CoutP][kC3PS]
    const int n = blockIdx.z, r0 = blockIdx.y * TR, c0 = blockIdx.x * 32;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = lane & 15, grp = lane >> 4;
    const int h = wid & 1, rg = wid >> 1;
    const size_t img = (size_t)n * H * W;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int cc0 = 0; cc0 < Cin; cc0 += kC3Chunk) {
        __syncthreads();  // the previous chunk is done with the LDS
        stage16<(NWIN + 255) / 256>(
            NWIN,
            [&](int it) -> const u16 * {
                const int px = it >> 2, ci = cc0 + (it & 3) * 8;
                const int hr = px / HC, hc = px - hr * HC;
                const int rr = r0 - 1 + hr, cc = c0 - 1 + hc;
                if (rr < 0 || rr >= H || cc < 0 || cc >= W || ci >= Cin) return nullptr;
                return X + (img + (size_t)rr * W + cc) * Cin + ci;
            },
            [&](int it) { return win + (it >> 2) * kC3PS + (it & 3) * 8; });
        stage16<(NWTS + 255) / 256>(
            NWTS,
            [&](int it) -> const u16 * {
                const int row = it >> 2, ci = cc0 + (it & 3) * 8;  // row = tap CoutP + co
                return ci < Cin ? Wk + (size_t)row * Cin + ci : nullptr;
            },
            [&](int it) { return wts + (it >> 2) * kC3PS + (it & 3) * 8; });
        __syncthreads();
#pragma unroll
        for (int dc = 0; dc < 3; ++dc) {
            Frag a[MT + 2];
#pragma unroll
            for (int q = 0; q < MT + 2; ++q)
                a[q].u = *(const uint4 *)(win + ((rg * MT + q) * HC + 16 * h + m + dc) * kC3PS +
                                          8 * grp);
#pragma unroll
            for (int dr = 0; dr < 3; ++dr) {
                Frag b[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    b[t].u = *(const uint4 *)(wts + ((3 * dr + dc) * CoutP + 16 * t + m) * kC3PS +
                                              8 * grp);
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i + dr].v, b[t].v,
                                                                            acc[i][t], 0, 0, 0);
            }
        }
    }
    // epilogue: D[pixel 4 grp + q of the wave's row i][co = 16 t + m], through
    // LDS [pixel][co] (pixel = row * 32 + column within the tile)
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + m;
        const float bb = (bias && co < Cout) ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int pbase = (rg * MT + i) * 32 + 16 * h + 4 * grp;
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
    conv_store_tile<CoutP>(lds_raw, Y, mask, img, r0, c0, TR, H, W, Cout, out_f32);
}

// ----------------------------------------------------------- conv wgrad ---
// Partial weight and bias gradients of one chunk: a strip of kWgPix columns
// (from c0) of image n over rows [r0, r0 + 4 kst), in steps of four rows.
// dZ [N][H][W][Cout], X [N][H][W][Cin] (channel counts multiples of 8).
// Block = 4 waves; wave w takes row r + w of each step.  Per step the block
// stages, transposed into LDS ([channel][column], bf16):
//   dZ of the four rows, its TMS output-channel tiles,
//   X of rows r - 1 .. r + 4 (r .. r + 3 for 1x1), columns c0 - 1 ..
//   c0 + kWgPix + 2 (c0 .. for 1x1), its TNS input-channel tiles,
// zero outside the image.  For every k-step of 32 pixels a wave loads its
// dZ fragments once and, per kernel row dr and input tile, one 16-byte read
// of the X row plus the next dword, which give the column shifts 0, 1 and 2
// of the three taps (dr, dc); so each (tap, co tile, ci tile) product is one
// matrix-core step and dZ and X are read from HBM once per chunk (X rows
// r - 1 and r + 4 twice).  Threads t < 4 * 16 TMS of the ci-split 0 blocks
// also sum their dZ row and channel (the bias gradient).  At the end the
// four waves' sums are added in wave order through LDS and written to
// part[chunk][taps][CoutP][Cin], the bias to part[chunk][len + co] (len =
// taps CoutP Cin): every chunk's row is written whole by its split blocks.
// blockIdx.x = chunk * nsplit + split, split = sm * nsn + sn (co tiles sm
// TMS.., ci tiles sn TNS..), chunk = strip * nrc + row chunk.
constexpr int kWgPix = 64;
constexpr int kWgLD = kWgPix + 8;  // bf16 row stride of the staged arrays

__host__ __device__ constexpr int wg_xrows(int ks) { return ks == 3 ? 6 : 4; }

template <int KS, int TMS, int TNS>
__global__ __launch_bounds__(256, 2) void k_wgrad(const u16 *__restrict__ dZ,
                                               const u16 *__restrict__ X,
                                               float *__restrict__ part, int H, int W, int Cin,
                                               int Cout, int nstrip, int nrc, int kst, int nsn,
                                               int nsplit, size_t len, size_t pstride)
{
    constexpr int T = KS * KS, XR = wg_xrows(KS), ZC = 16 * TMS, XC = 16 * TNS;
    constexpr int halo = KS == 3 ? 1 : 0;
    constexpr int K4X = (kWgPix + 4 * halo) / 4;  // 4-column groups of a staged X row
    extern __shared__ __align__(16) unsigned char lds_raw[];
    u16 *sZ = (u16 *)lds_raw;           // [4][ZC][kWgLD]
    u16 *sX = sZ + 4 * ZC * kWgLD;      // [XR][XC][kWgLD]: element k is column c0 - halo + k
    const int split = blockIdx.x % nsplit, chunk = blockIdx.x / nsplit;
    const int sm = split / nsn, sn = split - sm * nsn;
    const int rc = chunk % nrc, strip = chunk / nrc;
    const int n = strip / nstrip, c0 = (strip - n * nstrip) * kWgPix;
    const int co0 = sm * ZC, ci0 = sn * XC;
    const int CoutP = (Cout + 15) / 16 * 16;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = lane & 15, grp = lane >> 4;
    const size_t img = (size_t)n * H * W;
    const bool bias = sn == 0;
    f32x4 acc[T][TMS][TNS];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int i = 0; i < TMS; ++i)
#pragma unroll
            for (int j = 0; j < TNS; ++j) acc[t][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    constexpr int zitems = 4 * (kWgPix / 4) * (ZC / 8), xitems = XR * K4X * (XC / 8);
    constexpr int NIT = (zitems + xitems + 255) / 256;  // staging items per thread
    // Staging item it = threadIdx.x + 256 q: four pixels by eight channels of
    // dZ (it < zitems) or X.  A step's loads are unconditional (a pixel or
    // channel outside the tensor reads its first element and is stored as
    // zero), so they are in flight together, and the next step's loads go
    // out before this step's matrix-core work.
    uint4 sv[NIT][4];
    unsigned sok[NIT];
    auto stage_load = [&](int r) {
#pragma unroll
        for (int qi = 0; qi < NIT; ++qi) {
            const int it = threadIdx.x + 256 * qi;
            unsigned ok = 0;
            if (it < zitems) {
                constexpr int per_row = (kWgPix / 4) * (ZC / 8);
                const int q = it / per_row, rem = it - q * per_row;
                const int px4 = rem / (ZC / 8), o8 = (rem - px4 * (ZC / 8)) * 8;
                const int rr = r + q, co = co0 + o8;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int cc = c0 + 4 * px4 + u;
                    const bool in = rr < H && cc < W && co < Cout;
                    ok |= (unsigned)in << u;
                    sv[qi][u] = *(const uint4 *)(dZ + (in ? (img + (size_t)rr * W + cc) * Cout + co : 0));
                }
            } else {
                constexpr int per_row = K4X * (XC / 8);
                const int jj = it < zitems + xitems ? it - zitems : 0;
                const int q = jj / per_row, rem = jj - q * per_row;
                const int k4 = rem / (XC / 8), o8 = (rem - k4 * (XC / 8)) * 8;
                const int rr = r - halo + q, ci = ci0 + o8;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int cc = c0 - halo + 4 * k4 + u;
                    const bool in = it < zitems + xitems && rr >= 0 && rr < H && cc >= 0 &&
                                    cc < W && ci < Cin;
                    ok |= (unsigned)in << u;
                    sv[qi][u] = *(const uint4 *)(X + (in ? (img + (size_t)rr * W + cc) * Cin + ci : 0));
                }
            }
            sok[qi] = ok;
        }
    };
    auto stage_store = [&]() {
#pragma unroll
        for (int qi = 0; qi < NIT; ++qi) {
            const int it = threadIdx.x + 256 * qi;
            if (it >= zitems + xitems) break;
            u16 *dst;
            if (it < zitems) {
                constexpr int per_row = (kWgPix / 4) * (ZC / 8);
                const int q = it / per_row, rem = it - q * per_row;
                const int px4 = rem / (ZC / 8), o8 = (rem - px4 * (ZC / 8)) * 8;
                dst = sZ + (size_t)(q * ZC + o8) * kWgLD + 4 * px4;
            } else {
                constexpr int per_row = K4X * (XC / 8);
                const int jj = it - zitems;
                const int q = jj / per_row, rem = jj - q * per_row;
                const int k4 = rem / (XC / 8), o8 = (rem - k4 * (XC / 8)) * 8;
                dst = sX + (size_t)(q * XC + o8) * kWgLD + 4 * k4;
            }
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = (sok[qi] >> u) & 1u ? sv[qi][u] : make_uint4(0, 0, 0, 0);
            const u16 *e0 = (const u16 *)&v[0], *e1 = (const u16 *)&v[1];
            const u16 *e2 = (const u16 *)&v[2], *e3 = (const u16 *)&v[3];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                uint2 w;
                w.x = (uint32_t)e0[e] | ((uint32_t)e1[e] << 16);
                w.y = (uint32_t)e2[e] | ((uint32_t)e3[e] << 16);
                *(uint2 *)(dst + (size_t)e * kWgLD) = w;
            }
        }
    };
    const int st0 = rc * kst, nst = min(kst, (H + 3) / 4 - st0);
    stage_load(st0 * 4);
    for (int st = 0; st < nst; ++st) {
        __syncthreads();  // the previous step is done with the LDS
        stage_store();
        __syncthreads();
        if (st + 1 < nst) stage_load((st0 + st + 1) * 4);
        if (bias && (int)threadIdx.x < 4 * ZC) {  // row t / ZC, channel t % ZC
            const u16 *zr = sZ + (size_t)threadIdx.x * kWgLD;
#pragma unroll
            for (int k = 0; k < kWgPix; k += 8) {
                const uint4 v = *(const uint4 *)(zr + k);
                const u16 *e = (const u16 *)&v;
#pragma unroll
                for (int q = 0; q < 8; ++q) bsum += bf2f(e[q]);
            }
        }
#pragma unroll
        for (int ks = 0; ks < kWgPix; ks += 32) {
            Frag a[TMS];
#pragma unroll
            for (int i = 0; i < TMS; ++i)
                a[i].u = *(const uint4 *)(sZ + (size_t)(wid * ZC + i * 16 + m) * kWgLD + 8 * grp + ks);
#pragma unroll
            for (int dr = 0; dr < KS; ++dr)
#pragma unroll
                for (int j = 0; j < TNS; ++j) {
                    const u16 *xr = sX + (size_t)((wid + dr) * XC + j * 16 + m) * kWgLD + 8 * grp + ks;
                    Frag b0;
                    b0.u = *(const uint4 *)xr;
                    if constexpr (KS == 1) {
#pragma unroll
                        for (int i = 0; i < TMS; ++i)
                            acc[0][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i].v, b0.v,
                                                                                   acc[0][i][j], 0, 0, 0);
                    } else {
                        const uint4 v = b0.u;
                        const uint32_t nx = *(const uint32_t *)(xr + 8);
                        Frag b1, b2;
                        b1.u = make_uint4(__builtin_amdgcn_alignbit(v.y, v.x, 16),
                                          __builtin_amdgcn_alignbit(v.z, v.y, 16),
                                          __builtin_amdgcn_alignbit(v.w, v.z, 16),
                                          __builtin_amdgcn_alignbit(nx, v.w, 16));
                        b2.u = make_uint4(v.y, v.z, v.w, nx);
#pragma unroll
                        for (int i = 0; i < TMS; ++i) {
                            acc[3 * dr][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                a[i].v, b0.v, acc[3 * dr][i][j], 0, 0, 0);
                            acc[3 * dr + 1][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                a[i].v, b1.v, acc[3 * dr + 1][i][j], 0, 0, 0);
                            acc[3 * dr + 2][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                a[i].v, b2.v, acc[3 * dr + 2][i][j], 0, 0, 0);
                        }
                    }
                }
        }
    }
    // the waves' sums, added in wave order, one tap at a time
    float *red = (float *)lds_raw;  // [3][TMS][TNS][4][64]
    float *dst = part + (size_t)chunk * pstride;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        __syncthreads();
        if (wid > 0) {
#pragma unroll
            for (int i = 0; i < TMS; ++i)
#pragma unroll
                for (int j = 0; j < TNS; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        red[((((wid - 1) * TMS + i) * TNS + j) * 4 + q) * 64 + lane] = acc[t][i][j][q];
        }
        __syncthreads();
        if (wid == 0) {
#pragma unroll
            for (int i = 0; i < TMS; ++i)
#pragma unroll
                for (int j = 0; j < TNS; ++j) {
                    const int ci = ci0 + j * 16 + m;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float v = acc[t][i][j][q];
#pragma unroll
                        for (int w = 0; w < 3; ++w) v += red[(((w * TMS + i) * TNS + j) * 4 + q) * 64 + lane];
                        if (ci < Cin)
                            dst[((size_t)t * CoutP + co0 + i * 16 + 4 * grp + q) * Cin + ci] = v;
                    }
                }
        }
    }
    if (bias) {
        __syncthreads();
        if ((int)threadIdx.x < 4 * ZC) red[threadIdx.x] = bsum;
        __syncthreads();
        if ((int)threadIdx.x < ZC) {
            const int c = threadIdx.x;
            dst[len + co0 + c] = ((red[c] + red[ZC + c]) + red[2 * ZC + c]) + red[3 * ZC + c];
        }
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

// The sum of the nseg segments in segment order: element i < len0 to out0[i],
// the rest to out1[i - len0].
__global__ __launch_bounds__(256) void k_sum_out(const float *__restrict__ seg,
                                                 float *__restrict__ out0, float *__restrict__ out1,
                                                 int nseg, size_t len0, size_t len)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int q = 0; q < nseg; ++q) s += seg[(size_t)q * len + i];
    if (i < len0) out0[i] = s;
    else out1[i - len0] = s;
}

// Segments for summing nchunk partials of len values: enough blocks to
// spread the reads over the GPU, at least 4 chunks per segment and at most
// 64 segments (the second pass adds them one after another).
inline int sum_segments(int nchunk, size_t len)
{
    const size_t bx = (len + 255) / 256;
    size_t S = (2048 + bx - 1) / bx;
    S = std::min<size_t>(S, (size_t)std::max(1, nchunk / 4));
    S = std::min<size_t>(S, 64);
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

// z = bf16(a + b) where y > 0, else 0 (a sum's gradient through a ReLU)
__global__ void k_add_relu_bwd(const u16 *__restrict__ a, const u16 *__restrict__ b,
                               const u16 *__restrict__ y, u16 *__restrict__ z, size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    z[i] = bf2f(y[i]) > 0.f ? f2bf(bf2f(a[i]) + bf2f(b[i])) : (u16)0;
}

__global__ void k_add_relu_bwd8(const uint4 *__restrict__ a, const uint4 *__restrict__ b,
                                const uint4 *__restrict__ y, uint4 *__restrict__ z, size_t n8)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n8) return;
    uint4 x = a[i], w = b[i], m = y[i], r;
    const u16 *ex = (const u16 *)&x, *ew = (const u16 *)&w, *em = (const u16 *)&m;
    u16 *er = (u16 *)&r;
#pragma unroll
    for (int q = 0; q < 8; ++q) er[q] = bf2f(em[q]) > 0.f ? f2bf(bf2f(ex[q]) + bf2f(ew[q])) : (u16)0;
    z[i] = r;
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

// z = (depth-to-space of t: C1 channels, s: C2 channels) in 8-channel pieces,
// one thread per piece of z; inverse: t and s from z
__global__ void k_shuffle_concat8(uint4 *__restrict__ t, uint4 *__restrict__ s,
                                  uint4 *__restrict__ z, int N, int Hin, int Win, int C1, int C2,
                                  int inverse)
{
    const int g1 = C1 / 8, g = (C1 + C2) / 8;
    const int H = 2 * Hin, W = 2 * Win;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)N * H * W * g) return;
    const size_t p = i / g;
    const int c = (int)(i - p * g);
    uint4 *src;
    if (c < g1) {
        const int w = (int)(p % W), h = (int)((p / W) % H), n = (int)(p / ((size_t)W * H));
        src = t + (((size_t)n * Hin + h / 2) * Win + w / 2) * (4 * g1) +
              ((h % 2) * 2 + (w % 2)) * g1 + c;
    } else {
        src = s + p * (g - g1) + (c - g1);
    }
    if (!inverse) z[i] = *src;
    else *src = z[i];
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

static dect_status conv_fwd_launch(const void *x, const void *w, const float *bias,
                                   const void *mask, void *y, int32_t N, int32_t H, int32_t W,
                                   int32_t Cin, int32_t Cout, int32_t ksize, int32_t relu,
                                   int32_t out_f32, void *stream)
{
    if (!x || !w || !y || N <= 0 || H <= 0 || W <= 0 || Cin <= 0 || Cout <= 0)
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd: bad arguments");
    if (Cin % 8 != 0 || Cout > 256 || (ksize != 1 && ksize != 3))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd: Cin % 8, Cout <= 256, ksize in {1,3}");
    if (mask && (((uintptr_t)mask & 15) != 0))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd: mask must be 16-byte aligned");
    const int NT = (Cout + 15) / 16;
    hipStream_t s = (hipStream_t)stream;
    const u16 *X = (const u16 *)x, *Wk = (const u16 *)w, *Mk = (const u16 *)mask;
    if (ksize == 3 && conv3_use(NT, Cin)) {
        switch (NT) {
#define CASE3(nt)                                                                           \
    case nt: {                                                                              \
        constexpr int tr = 2 * conv3_mt(nt);                                                \
        hipLaunchKernelGGL(k_conv3<nt>, dim3((W + 31) / 32, (H + tr - 1) / tr, N), dim3(256), \
                           (unsigned)conv3_lds(nt, out_f32), s, X, Wk, bias, y, H, W, Cin,  \
                           Cout, relu, out_f32, Mk);                                        \
    } break;
            CASE3(1) CASE3(2) CASE3(3) CASE3(4) CASE3(5) CASE3(6) CASE3(7) CASE3(8)
#undef CASE3
            default: return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd: no 3x3 kernel for this width");
        }
        NN_HIP(hipGetLastError());
        return DECT_OK;
    }
    switch (NT) {
#define CASE(nt)                                                                         \
    case nt: {                                                                           \
        dim3 grid((W + 31) / 32, (H + 2 * conv_mt(nt) - 1) / (2 * conv_mt(nt)), N);      \
        hipLaunchKernelGGL(k_conv_fwd<nt>, grid, dim3(256),                                \
                           (unsigned)conv_fwd_lds(nt, Cin, ksize, out_f32), s, X, Wk, bias, y, \
                           H, W, Cin, Cout, ksize, relu, out_f32, Mk);                   \
    } break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    NN_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status dect_nn_conv_fwd(const void *x, const void *w, const float *bias, void *y, int32_t N,
                             int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                             int32_t relu, int32_t out_f32, void *stream)
{
    return conv_fwd_launch(x, w, bias, nullptr, y, N, H, W, Cin, Cout, ksize, relu, out_f32,
                           stream);
}

dect_status dect_nn_conv_fwd_masked(const void *x, const void *w, const float *bias,
                                    const void *mask, void *y, int32_t N, int32_t H, int32_t W,
                                    int32_t Cin, int32_t Cout, int32_t ksize, int32_t relu,
                                    int32_t out_f32, void *stream)
{
    if (!mask) return nn_fail(DECT_ERR_INVALID_ARG, "conv_fwd_masked: null mask");
    return conv_fwd_launch(x, w, bias, mask, y, N, H, W, Cin, Cout, ksize, relu, out_f32, stream);
}

// Tiles per weight-gradient block: TMS output-channel x TNS input-channel
// tiles (taps x TMS x TNS accumulators of four floats per lane: at most 108
// for 3x3; staged rows within 64 KB of LDS for 1x1), the first entry of a
// fixed list that divides the layer's tile counts.  For 3x3, two tiles per
// block measured fastest: (2, 2) needs 226 registers (two waves per SIMD),
// (2, 1) about 140 (three), which outweighs reading dZ once per input tile
// pair instead of once; (1, 1) reads both operands too often.
struct WgTiles {
    int tms, tns;
};

static WgTiles wgrad_tiles(int ks, int TM, int TN)
{
    static const WgTiles k3[] = {{2, 1}, {3, 1}, {1, 2}, {1, 1}};
    static const WgTiles k1[] = {{4, 2}, {3, 3}, {2, 3}, {3, 2}, {4, 1}, {2, 2},
                                 {3, 1}, {1, 3}, {2, 1}, {1, 2}, {1, 1}};
    const WgTiles *list = ks == 3 ? k3 : k1;
    const int n = ks == 3 ? 4 : 11;
    for (int i = 0; i < n; ++i)
        if (TM % list[i].tms == 0 && TN % list[i].tns == 0) return list[i];
    return {1, 1};
}

struct WgradPlan {
    int tms, tns, nsm, nsn, nstrip, nrc, kst, nchunk, nseg;
    size_t lds, len, pstride;
};

static const void *wgrad_kernel(int ks, int tms, int tns)
{
#define WGK(k, a, b) \
    if (ks == k && tms == a && tns == b) return (const void *)k_wgrad<k, a, b>;
    WGK(3, 3, 1) WGK(3, 2, 1) WGK(3, 1, 2) WGK(3, 1, 1)
    WGK(1, 4, 2) WGK(1, 3, 3) WGK(1, 2, 3) WGK(1, 3, 2) WGK(1, 4, 1) WGK(1, 2, 2)
    WGK(1, 3, 1) WGK(1, 1, 3) WGK(1, 2, 1) WGK(1, 1, 2) WGK(1, 1, 1)
#undef WGK
    return nullptr;
}

// Blocks of a tiling's kernel resident on the current device at once (its
// compute units times the blocks per unit its registers and LDS allow),
// queried once per device and tiling.
static int wgrad_resident(int ks, int tms, int tns, size_t lds)
{
    static std::mutex mu;
    static std::map<std::array<int, 4>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const std::array<int, 4> key{dev, ks, tms, tns};
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    const void *k = wgrad_kernel(ks, tms, tns);
    if (!k || dev < 0 ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu <= 0 || cus <= 0) {
        (void)hipGetLastError();
        per_cu = 2;
        cus = 256;
    }
    return cache[key] = per_cu * cus;
}

static WgradPlan wgrad_plan(int N, int H, int W, int Cin, int Cout, int ksize)
{
    WgradPlan q;
    const int CoutP = (Cout + 15) / 16 * 16, CinP = (Cin + 15) / 16 * 16;
    const WgTiles t = wgrad_tiles(ksize, CoutP / 16, CinP / 16);
    q.tms = t.tms;
    q.tns = t.tns;
    q.nsm = CoutP / 16 / t.tms;
    q.nsn = CinP / 16 / t.tns;
    const int nsplit = q.nsm * q.nsn;
    q.nstrip = (W + kWgPix - 1) / kWgPix;
    const size_t RG = (size_t)(H + 3) / 4;  // steps of four rows per strip
    const size_t strips = (size_t)N * q.nstrip;
    q.len = (size_t)ksize * ksize * CoutP * Cin;
    q.pstride = q.len + CoutP;
    const size_t stage =
        ((size_t)4 * 16 * t.tms + (size_t)wg_xrows(ksize) * 16 * t.tns) * kWgLD * sizeof(u16);
    const size_t red = (size_t)3 * t.tms * t.tns * 4 * 64 * sizeof(float);
    q.lds = std::max(stage, red);
    // one round of resident blocks, fewer while the partials would outweigh
    // twice the layer's own bytes
    const size_t target = (size_t)wgrad_resident(ksize, t.tms, t.tns, q.lds);
    size_t kst = std::max<size_t>(1, (strips * RG * nsplit + target - 1) / target);
    const double in_bytes = (double)N * H * W * (Cin + Cout) * 2;
    while (kst < RG && (double)strips * ((RG + kst - 1) / kst) * q.pstride * 4 > 2.0 * in_bytes)
        kst *= 2;
    kst = std::min(kst, RG);
    q.kst = (int)kst;
    q.nrc = (int)((RG + kst - 1) / kst);
    q.nchunk = (int)(strips * q.nrc);
    q.nseg = sum_segments(q.nchunk, q.pstride);
    return q;
}

size_t dect_nn_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                               int32_t ksize)
{
    if (N <= 0 || H <= 0 || W <= 0 || Cin <= 0 || Cout <= 0 || (ksize != 1 && ksize != 3))
        return 0;
    const WgradPlan q = wgrad_plan(N, H, W, Cin, Cout, ksize);
    return ((size_t)q.nchunk + q.nseg) * q.pstride * sizeof(float);
}

dect_status dect_nn_conv_wgrad(const void *dz, const void *x, float *dw, float *db, int32_t N,
                               int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t ksize,
                               void *workspace, size_t ws_bytes, void *stream)
{
    if (!dz || !x || !dw || !db || !workspace || N <= 0 || H <= 0 || W <= 0)
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: bad arguments");
    if (Cin <= 0 || Cout <= 0 || Cin % 8 != 0 || Cout % 8 != 0 || Cin > 256 || Cout > 256 ||
        (ksize != 1 && ksize != 3))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: Cin, Cout % 8 and <= 256");
    if (ws_bytes < dect_nn_wgrad_workspace(N, H, W, Cin, Cout, ksize))
        return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: workspace too small");
    const WgradPlan q = wgrad_plan(N, H, W, Cin, Cout, ksize);
    const size_t nblk = (size_t)q.nchunk * q.nsm * q.nsn;
    if (nblk > 0x7fffffffu) return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: problem too large");
    float *part = (float *)workspace;
    float *seg = part + (size_t)q.nchunk * q.pstride;
    hipStream_t s = (hipStream_t)stream;
    const u16 *Z = (const u16 *)dz, *Xp = (const u16 *)x;
    bool launched = false;
#define WG(ks, a, b)                                                                          \
    if (!launched && ksize == ks && q.tms == a && q.tns == b) {                               \
        hipLaunchKernelGGL((k_wgrad<ks, a, b>), dim3((unsigned)nblk), dim3(256), q.lds, s, Z, \
                           Xp, part, H, W, Cin, Cout, q.nstrip, q.nrc, q.kst, q.nsn,          \
                           q.nsm * q.nsn, q.len, q.pstride);                                  \
        launched = true;                                                                      \
    }
    WG(3, 3, 1) WG(3, 2, 1) WG(3, 1, 2) WG(3, 1, 1)
    WG(1, 4, 2) WG(1, 3, 3) WG(1, 2, 3) WG(1, 3, 2) WG(1, 4, 1) WG(1, 2, 2)
    WG(1, 3, 1) WG(1, 1, 3) WG(1, 2, 1) WG(1, 1, 2) WG(1, 1, 1)
#undef WG
    if (!launched) return nn_fail(DECT_ERR_INVALID_ARG, "conv_wgrad: no kernel for this tiling");
    NN_HIP(hipGetLastError());
    const int L = (q.nchunk + q.nseg - 1) / q.nseg;
    hipLaunchKernelGGL(k_sum_seg, dim3(blocks(q.pstride), q.nseg), dim3(256), 0, s, part, seg,
                       q.nchunk, q.pstride, L);
    hipLaunchKernelGGL(k_sum_out, dim3(blocks(q.pstride)), dim3(256), 0, s, seg, dw, db, q.nseg,
                       q.len, q.pstride);
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

dect_status dect_nn_shuffle_concat(void *t, void *s, void *z, int32_t N, int32_t Hin, int32_t Win,
                                   int32_t C1, int32_t C2, int32_t inverse, void *stream)
{
    if (!t || !s || !z || N <= 0 || Hin <= 0 || Win <= 0 || C1 <= 0 || C2 <= 0 ||
        C1 % 8 != 0 || C2 % 8 != 0 || !aligned16(t) || !aligned16(s) || !aligned16(z))
        return nn_fail(DECT_ERR_INVALID_ARG,
                       "shuffle_concat: channels must be positive multiples of 8, pointers "
                       "16-byte aligned");
    const size_t pieces = (size_t)N * 4 * Hin * Win * ((C1 + C2) / 8);
    hipLaunchKernelGGL(k_shuffle_concat8, dim3(blocks(pieces)), dim3(256), 0,
                       (hipStream_t)stream, (uint4 *)t, (uint4 *)s, (uint4 *)z, N, Hin, Win, C1,
                       C2, inverse);
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

dect_status dect_nn_add_relu_bwd(const void *a, const void *b, const void *y, void *z, size_t n,
                                 void *stream)
{
    if (n == 0) return DECT_OK;
    if (!a || !b || !y || !z) return nn_fail(DECT_ERR_INVALID_ARG, "add_relu_bwd: null argument");
    if (n % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(y) && aligned16(z))
        hipLaunchKernelGGL(k_add_relu_bwd8, dim3(blocks(n / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint4 *)a, (const uint4 *)b, (const uint4 *)y, (uint4 *)z, n / 8);
    else
        hipLaunchKernelGGL(k_add_relu_bwd, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                           (const u16 *)a, (const u16 *)b, (const u16 *)y, (u16 *)z, n);
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
