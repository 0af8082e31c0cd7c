// Learned MB localiser: a small 2D CNN on the filtered projection envelope.
// The paper points to deep-learning localisation as the way past NCC on dense
// MB populations (Section IV); this is the learned alternative to the NCC step.
//   input   I / max_frame(I), one channel, H x W (the plane grid)
//   layers  conv3x3 1 -> 32 + ReLU, then 5 x conv3x3 32 -> 32 + ReLU (zero pad 1)
//   head    1x1 conv 32 -> 64, depth-to-space x8: a heatmap on a grid 8x finer
//   loss    mean squared error against T(q) = max_MB exp(-|q - (8 (x + 1/2) - 1/2)|^2 / 2)
//   update  Adam on FP32 master parameters
//   decode  3x3 local maxima of the heatmap (raster tie-break) at or above a threshold
//
// Activations are stored channel-innermost ([n][y][x][32]) in BF16 (product) or
// FP32 (reference precision); accumulation is FP32 in both.  The 32 -> 32
// convolutions and the head are matrix products on MFMA: 32 pixels of a row x
// 32 output channels per wave, K = 9 taps x 32 input channels
// (v_mfma_f32_32x32x16_bf16, or v_mfma_f32_32x32x2f32).  The data gradient of
// a convolution is the same kernel with transposed, flipped weights and the
// ReLU mask of the layer below.  Inference fuses the head with the decode, so
// the 64-values-per-pixel heatmap never reaches HBM.
//
// Flat FP32 parameter vector:
//   w0 [32][1][3][3], b0 [32], then for l = 1..5: wl [32][32][3][3], bl [32],
//   wh [64][32], bh [64]          (48,672 values)
#include "common.h"

#include <math.h>
#include <algorithm>

namespace ulm {

constexpr int kC = 32;           // channels
constexpr int kL = 6;            // conv layers
constexpr int kR = 8;            // heatmap upsampling
constexpr int kR2 = kR * kR;     // head outputs per pixel
constexpr int kW0 = kC * 9, kB0 = kC;
constexpr int kWl = kC * kC * 9, kBl = kC;
constexpr int kWh = kR2 * kC, kBh = kR2;
constexpr int kParams = kW0 + kB0 + (kL - 1) * (kWl + kBl) + kWh + kBh;
static_assert(kParams == ULM_CNN_PARAMS, "parameter count");

__host__ __device__ constexpr int off_w(int l) { return l == 0 ? 0 : kW0 + kB0 + (l - 1) * (kWl + kBl); }
__host__ __device__ constexpr int off_b(int l) { return l == 0 ? kW0 : off_w(l) + kWl; }
__host__ __device__ constexpr int off_wh() { return kW0 + kB0 + (kL - 1) * (kWl + kBl); }
__host__ __device__ constexpr int off_bh() { return off_wh() + kWh; }

constexpr int kTileRows = 4, kTileCols = 32;   // conv tile: one 32-pixel row per wave
constexpr int kHeadPx = 128;                   // pixels per head-gradient chunk
constexpr int kMaxPartials = 256;              // work-groups of a weight-gradient pass

typedef __bf16 bf16;
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// LDS strides (elements) chosen so that the 32 lanes of a half-wave hit distinct banks
template <typename T> struct Lds;
template <> struct Lds<bf16> { static constexpr int px = 40, w = 9 * kC + 8, wh = 40; };
template <> struct Lds<float> { static constexpr int px = 33, w = 9 * kC + 1, wh = 33; };

__device__ inline float tof(float x) { return x; }
__device__ inline float tof(bf16 x) { return (float)x; }
template <typename T> __device__ inline T fromf(float x) { return (T)x; }

// ----------------------------------------------------------------- small kernels
__global__ void cnn_fill_kernel(int *__restrict__ p, size_t n, int v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void cnn_status_clear_kernel(int *status, int bits) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAnd(status, ~bits);
}

// wm [5][32 out][9 tap][32 in], wt [5][32 in][9 (8 - tap)][32 out], both in T
template <typename T>
__global__ void cnn_prepare_kernel(const float *__restrict__ p, T *__restrict__ wm, T *__restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (kL - 1) * kWl) return;
    const int l = i / kWl, r = i % kWl;
    const int o = r / (kC * 9), c = (r / 9) % kC, tap = r % 9;      // source [o][c][tap]
    const T v = fromf<T>(p[off_w(l + 1) + r]);
    wm[(size_t)l * kWl + (o * 9 + tap) * kC + c] = v;
    wt[(size_t)l * kWl + (c * 9 + (8 - tap)) * kC + o] = v;
}

// |v| with one fixed rounding sequence (im^2 fused onto the rounded re^2), so
// every kernel that forms the network input gets the same bits
__device__ inline float cnn_mag(float2 v) { return sqrtf(fmaf(v.y, v.y, v.x * v.x)); }

// x0[n][i] = |P[n0 + n][i]| / max over that image of |P|   (0 for an all-zero image)
__global__ __launch_bounds__(256) void cnn_input_kernel(const float2 *__restrict__ P,
                                                        const float *__restrict__ fmax,
                                                        float *__restrict__ x0, int npix, int n0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (i >= npix) return;
    const float2 v = P[(size_t)(n0 + n) * npix + i];
    const float m = fmax[n0 + n];
    x0[(size_t)n * npix + i] = m > 0.f ? cnn_mag(v) / m : 0.f;
}

// ----------------------------------------------------------------- layer 0 (1 -> 32)
template <typename T>
__global__ __launch_bounds__(256) void cnn_conv0_kernel(const float *__restrict__ x0,
                                                        const float *__restrict__ p,
                                                        T *__restrict__ a1, int H, int W, size_t npx)
{
    __shared__ float w[kW0 + kB0];
    for (int e = threadIdx.x; e < kW0 + kB0; e += blockDim.x) w[e] = p[e];
    __syncthreads();
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npx) return;
    const int x = idx % W, y = (idx / W) % H;
    const size_t n = idx / ((size_t)W * H);
    float in[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int yy = y + dy - 1, xx = x + dx - 1;
            in[dy * 3 + dx] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                                  ? x0[(n * H + yy) * W + xx] : 0.f;
        }
    // 32 outputs of this pixel, written as 16-byte vectors
    T res[kC];
#pragma unroll
    for (int o = 0; o < kC; ++o) {
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) s = fmaf(w[o * 9 + t], in[t], s);
        res[o] = fromf<T>(fmaxf(s + w[kW0 + o], 0.f));
    }
    uint4 *dst = reinterpret_cast<uint4 *>(a1 + idx * kC);
#pragma unroll
    for (int q = 0; q < (int)(kC * sizeof(T) / 16); ++q) dst[q] = reinterpret_cast<const uint4 *>(res)[q];
}

// ----------------------------------------------------------------- 32 -> 32 conv
// out[n][y][x][o] = epi( sum_{tap, c} w[o][tap][c] in[n][y + dy - 1][x + dx - 1][c] )
// MASK = false: + bias, ReLU (forward).  MASK = true: zero where mask <= 0 (data gradient).
// Persistent: each work-group stages the layer's weights in LDS once and then
// walks the 4 x 32 pixel tiles blockIdx.x, blockIdx.x + gridDim.x, ...; the
// results go through a per-wave LDS transpose so every lane writes whole
// 16-byte channel groups.
template <typename T>
constexpr int kEpiStride = kC + 16 / (int)sizeof(T);     // padded channels per staged pixel

template <typename T, bool MASK>
__global__ __launch_bounds__(256) void cnn_conv_kernel(const T *__restrict__ in,
                                                       const T *__restrict__ w,
                                                       const float *__restrict__ bias,
                                                       const T *__restrict__ mask,
                                                       T *__restrict__ out, int H, int W, int B)
{
    constexpr int PS = Lds<T>::px, WS = Lds<T>::w, TC = kTileCols + 2, ES = kEpiStride<T>;
    constexpr int VEC = 16 / (int)sizeof(T);                // elements per 16-byte vector
    __shared__ __attribute__((aligned(16))) T tile[(kTileRows + 2) * TC * PS];
    __shared__ __attribute__((aligned(16))) T wl[kC * WS];
    static_assert(4 * kTileCols * ES <= (kTileRows + 2) * TC * PS, "epilogue fits in the tile");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if constexpr (sizeof(T) == 2) {
        for (int e = t; e < kC * 36; e += 256) {
            const int o = e / 36, q = e % 36;
            *reinterpret_cast<uint4 *>(&wl[o * WS + q * 8]) = reinterpret_cast<const uint4 *>(w)[e];
        }
    } else {
        for (int e = t; e < kC * 9 * kC; e += 256) wl[(e / (9 * kC)) * WS + e % (9 * kC)] = w[e];
    }
    const int tx = cdiv(W, kTileCols), ty = cdiv(H, kTileRows);
    const long ntiles = (long)tx * ty * B;
    const int i32 = lane & 31, hk = lane >> 5;
    const float b = MASK ? 0.f : bias[i32];
    for (long tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const int n = (int)(tl / ((long)tx * ty)), y0 = (int)((tl / tx) % ty) * kTileRows,
                  x0 = (int)(tl % tx) * kTileCols;
        __syncthreads();       // the previous tile's readers are done with `tile`
        if constexpr (sizeof(T) == 2) {
            for (int e = t; e < (kTileRows + 2) * TC * 4; e += 256) {
                const int q = e & 3, px = (e >> 2) % TC, ry = (e >> 2) / TC;
                const int yy = y0 + ry - 1, xx = x0 + px - 1;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    v = reinterpret_cast<const uint4 *>(in + (((size_t)n * H + yy) * W + xx) * kC)[q];
                *reinterpret_cast<uint4 *>(&tile[(ry * TC + px) * PS + q * 8]) = v;
            }
        } else {
            for (int e = t; e < (kTileRows + 2) * TC * kC; e += 256) {
                const int c = e % kC, px = (e / kC) % TC, ry = e / (kC * TC);
                const int yy = y0 + ry - 1, xx = x0 + px - 1;
                tile[(ry * TC + px) * PS + c] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                                                    ? in[(((size_t)n * H + yy) * W + xx) * kC + c] : 0.f;
            }
        }
        __syncthreads();
        // two accumulation chains (the halves of each tap's channels), summed at
        // the end, so consecutive MFMAs do not wait on each other's results
        f32x16 acc2[2] = {{}, {}};
        if constexpr (sizeof(T) == 2) {
            // the next tap's operands are read while this tap's MFMAs run
            bf16x8 av[2][2], bv[2][2];
            auto fetch = [&](int tap, int slot) {
                const int dy = tap / 3, dx = tap % 3;
                const T *arow = &tile[((wave + dy) * TC + i32 + dx) * PS];
                const T *brow = &wl[i32 * WS + tap * kC];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    av[slot][h] = *reinterpret_cast<const bf16x8 *>(arow + h * 16 + hk * 8);
                    bv[slot][h] = *reinterpret_cast<const bf16x8 *>(brow + h * 16 + hk * 8);
                }
            };
            fetch(0, 0);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                if (tap + 1 < 9) fetch(tap + 1, (tap + 1) & 1);
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    acc2[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[tap & 1][h], bv[tap & 1][h], acc2[h],
                                                                      0, 0, 0);
            }
        } else {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;
                const T *arow = &tile[((wave + dy) * TC + i32 + dx) * PS];
                const T *brow = &wl[i32 * WS + tap * kC];
#pragma unroll
                for (int s2 = 0; s2 < 16; ++s2)
                    acc2[s2 & 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(arow[2 * s2 + hk], brow[2 * s2 + hk],
                                                                        acc2[s2 & 1], 0, 0, 0);
            }
        }
        const f32x16 acc = acc2[0] + acc2[1];
        // lane holds D[8 (q / 4) + 4 hk + q % 4][i32]: pixel row of the tile, output channel i32;
        // the tile's LDS is reused to transpose the results (every wave is done reading it)
        __syncthreads();
        T *epw = tile + wave * kTileCols * ES;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int pr = 8 * (q >> 2) + 4 * hk + (q & 3);
            const float v = MASK ? acc[q] : fmaxf(acc[q] + b, 0.f);
            epw[pr * ES + i32] = fromf<T>(v);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);       // this wave's LDS writes have landed
        __builtin_amdgcn_wave_barrier();
        const int y = y0 + wave;
        if (y < H) {
            constexpr int NV = kTileCols * kC / VEC;     // 16-byte vectors per wave row
#pragma unroll
            for (int c = lane; c < NV; c += 64) {
                const int pr = c / (kC / VEC), g = c % (kC / VEC);
                const int x = x0 + pr;
                if (x < W) {
                    const size_t at = (((size_t)n * H + y) * W + x) * kC + g * VEC;
                    uint4 v = *reinterpret_cast<const uint4 *>(&epw[pr * ES + g * VEC]);
                    if constexpr (MASK) {
                        const uint4 mv = *reinterpret_cast<const uint4 *>(mask + at);
                        const T *mk = reinterpret_cast<const T *>(&mv);
                        T *vv = reinterpret_cast<T *>(&v);
#pragma unroll
                        for (int i = 0; i < VEC; ++i)
                            if (!(tof(mk[i]) > 0.f)) vv[i] = fromf<T>(0.f);
                    }
                    *reinterpret_cast<uint4 *>(out + at) = v;
                }
            }
        }
    }
}

// BF16 forward form of the 32 -> 32 convolution with taller tiles and the next
// tile's loads in flight: 8 x 32 output pixels per tile (two rows per wave, the
// B operands of a tap shared by both), the input tile (10 x 34 pixels) staged
// in one of two LDS buffers while the other is read, the next tile's channel
// vectors held in registers during the MFMAs.  Two barriers per tile.
constexpr int kCvRows = 8;

__global__ __launch_bounds__(256, 2) void cnn_conv_fwd_bf16_kernel(const bf16 *__restrict__ in,
                                                                   const bf16 *__restrict__ w,
                                                                   const float *__restrict__ bias,
                                                                   bf16 *__restrict__ out, int H, int W,
                                                                   int B)
{
    constexpr int PS = Lds<bf16>::px, WS = Lds<bf16>::w, TC = kTileCols + 2, TR = kCvRows + 2;
    constexpr int ES = kEpiStride<bf16>, VEC = 8;
    constexpr int NV = TR * TC * 4;                          // 16-byte vectors per input tile
    constexpr int NQ = (NV + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 tile[2][TR * TC * PS];
    __shared__ __attribute__((aligned(16))) bf16 wl[kC * WS];
    static_assert(4 * 2 * kTileCols * ES <= TR * TC * PS, "epilogue fits in a tile buffer");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int e = t; e < kC * 36; e += 256) {
        const int o = e / 36, q = e % 36;
        *reinterpret_cast<uint4 *>(&wl[o * WS + q * 8]) = reinterpret_cast<const uint4 *>(w)[e];
    }
    const int tx = cdiv(W, kTileCols), ty = cdiv(H, kCvRows);
    const long ntiles = (long)tx * ty * B;
    const int i32 = lane & 31, hk = lane >> 5;
    const float b = bias[i32];
    uint4 pre[NQ];
    auto load = [&](long tl) {
        const int n = (int)(tl / ((long)tx * ty)), y0 = (int)((tl / tx) % ty) * kCvRows,
                  x0 = (int)(tl % tx) * kTileCols;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + q * 256;
            const int q4 = e & 3, px = (e >> 2) % TC, ry = (e >> 2) / TC;
            const int yy = y0 + ry - 1, xx = x0 + px - 1;
            pre[q] = make_uint4(0, 0, 0, 0);
            if (e < NV && yy >= 0 && yy < H && xx >= 0 && xx < W)
                pre[q] = reinterpret_cast<const uint4 *>(in + (((size_t)n * H + yy) * W + xx) * kC)[q4];
        }
    };
    auto put = [&](int bufi) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + q * 256;
            if (e < NV) {
                const int q4 = e & 3, px = (e >> 2) % TC, ry = (e >> 2) / TC;
                *reinterpret_cast<uint4 *>(&tile[bufi][(ry * TC + px) * PS + q4 * 8]) = pre[q];
            }
        }
    };
    long tl = blockIdx.x;
    if (tl < ntiles) {
        load(tl);
        put(0);
    }
    __syncthreads();
    int cur = 0;
    for (; tl < ntiles; tl += gridDim.x) {
        const int n = (int)(tl / ((long)tx * ty)), y0 = (int)((tl / tx) % ty) * kCvRows,
                  x0 = (int)(tl % tx) * kTileCols;
        const long nxt = tl + gridDim.x;
        if (nxt < ntiles) load(nxt);
        // rows wave and wave + 4 of the tile; two accumulation chains per row
        f32x16 acc[2][2] = {{{}, {}}, {{}, {}}};
        const bf16 *tb = tile[cur];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            const bf16 *brow = &wl[i32 * WS + tap * kC];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(brow + h * 16 + hk * 8);
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const bf16 *arow = &tb[((wave + 4 * r + dy) * TC + i32 + dx) * PS];
                    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(arow + h * 16 + hk * 8);
                    acc[r][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[r][h], 0, 0, 0);
                }
            }
        }
        __syncthreads();          // every wave is done reading tile[cur]
        // lane holds D[8 (q / 4) + 4 hk + q % 4][i32]: pixel of the row, output channel i32;
        // tile[cur] is reused to transpose the results
        bf16 *epw = tile[cur] + wave * 2 * kTileCols * ES;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const f32x16 a = acc[r][0] + acc[r][1];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int pr = 8 * (q >> 2) + 4 * hk + (q & 3);
                epw[(r * kTileCols + pr) * ES + i32] = fromf<bf16>(fmaxf(a[q] + b, 0.f));
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);       // this wave's LDS writes have landed
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = y0 + wave + 4 * r;
            if (y >= H) continue;
            constexpr int NR = kTileCols * kC / VEC;       // 16-byte vectors per output row
#pragma unroll
            for (int c = lane; c < NR; c += 64) {
                const int pr = c / (kC / VEC), g = c % (kC / VEC);
                const int x = x0 + pr;
                if (x < W) {
                    const size_t at = (((size_t)n * H + y) * W + x) * kC + g * VEC;
                    *reinterpret_cast<uint4 *>(out + at) =
                        *reinterpret_cast<const uint4 *>(&epw[(r * kTileCols + pr) * ES + g * VEC]);
                }
            }
        }
        if (nxt < ntiles) put(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
}

// ----------------------------------------------------------------- head
// Stage the head weights (T, padded rows) and biases in LDS.
template <typename T>
__device__ inline void stage_head(const float *__restrict__ p, T *whs, float *bhs) {
    constexpr int WS = Lds<T>::wh;
    for (int e = threadIdx.x; e < kWh; e += blockDim.x) whs[(e / kC) * WS + e % kC] = fromf<T>(p[off_wh() + e]);
    for (int e = threadIdx.x; e < kBh; e += blockDim.x) bhs[e] = p[off_bh() + e];
}

// One wave: 32 pixels (lane i32 supplies pixel `px`, or none when px < 0) x 64
// head outputs.  acc[nb][q] = bh[32 nb + i32] + sum_c wh[32 nb + i32][c] a[pixel
// 8(q/4) + 4hk + q%4][c]: the MFMAs start from the bias, so every form of the
// head (layer by layer and fused) rounds the same sums.
template <typename T>
__device__ inline void head_group(const T *__restrict__ act, long px, const T *whs, const float *bhs,
                                  f32x16 acc[2]) {
    constexpr int WS = Lds<T>::wh;
    const int lane = threadIdx.x & 63, i32 = lane & 31, hk = lane >> 5;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const float b = bhs[nb * 32 + i32];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[nb][q] = b;
    }
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 a = {};
            if (px >= 0) a = *reinterpret_cast<const bf16x8 *>(act + px * kC + h * 16 + hk * 8);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(whs + (nb * 32 + i32) * WS + h * 16 + hk * 8);
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nb], 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float a = px >= 0 ? act[px * kC + 2 * s + hk] : 0.f;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, whs[(nb * 32 + i32) * WS + 2 * s + hk],
                                                               acc[nb], 0, 0, 0);
        }
    }
}

// logits[px][k] = bh[k] + sum_c wh[k][c] a6[px][c] (summed from the bias); 32 pixels per wave
template <typename T>
__global__ __launch_bounds__(256) void cnn_head_kernel(const T *__restrict__ a6,
                                                       const float *__restrict__ p,
                                                       float *__restrict__ logits, size_t npx)
{
    __shared__ __attribute__((aligned(16))) T whs[kR2 * Lds<T>::wh];
    __shared__ float bhs[kR2];
    stage_head<T>(p, whs, bhs);
    __syncthreads();
    const int lane = threadIdx.x & 63, i32 = lane & 31, hk = lane >> 5;
    const size_t base = ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
    if (base >= npx) return;
    const long mine = base + i32 < npx ? (long)(base + i32) : -1;
    f32x16 acc[2];
    head_group<T>(a6, mine, whs, bhs, acc);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const size_t px = base + 8 * (q >> 2) + 4 * hk + (q & 3);
            const int k = nb * 32 + i32;
            if (px < npx) logits[px * kR2 + k] = acc[nb][q];
        }
}

// heat[n][8y + i][8x + j] = logits[n][y][x][8i + j]
__global__ void cnn_d2s_kernel(const float *__restrict__ logits, float *__restrict__ heat, int H,
                               int W, size_t total)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int Wf = W * kR, Hf = H * kR;
    const int fx = e % Wf, fy = (e / Wf) % Hf;
    const size_t n = e / ((size_t)Wf * Hf);
    heat[e] = logits[((n * H + fy / kR) * W + fx / kR) * kR2 + (fy % kR) * kR + fx % kR];
}

// ----------------------------------------------------------------- fused head + decode
// One work-group per (image, band of kHdRows coarse rows).  For each chunk of
// 32 coarse columns the head runs once on the band's rows and the rows above
// and below it (coarse rows y0-1 .. y0+kHdRows, columns x0-1 .. x0+32), so every
// fine pixel of the band has its 8 fine neighbours in LDS.  Candidates: heat >=
// thr, above the neighbours earlier in fine raster order and not below the
// later ones.  Each coarse row's records are compacted in (coarse column, fine
// row, fine column) order into that row's staging slot.
constexpr int kHdRows = 4;

template <typename T>
__global__ __launch_bounds__(256, 2) void cnn_head_decode_kernel(
    const T *__restrict__ a6, const float *__restrict__ p, const float2 *__restrict__ P, float thr,
    int H, int W, int n0, int F, ulm_loc_t *__restrict__ staged, int *__restrict__ row_cnt,
    int row_cap, int *__restrict__ status)
{
    constexpr int HC = kTileCols + 2, HR = kHdRows + 2, NS = HR * HC;
    __shared__ __attribute__((aligned(16))) T whs[kR2 * Lds<T>::wh];
    __shared__ float bhs[kR2];
    __shared__ float hs[HR][HC][kR2 + 1];       // +1: the decode's 64 lanes (8 columns x 8 fine rows) hit 64 banks
    __shared__ int wave_tot[kHdRows][4];
    __shared__ int base_s[kHdRows];
    stage_head<T>(p, whs, bhs);
    if (threadIdx.x < kHdRows) base_s[threadIdx.x] = 0;
    __syncthreads();
    const int y0 = blockIdx.x * kHdRows, n = blockIdx.y, img = n0 + n;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i32 = lane & 31, hk = lane >> 5;
    const T *act = a6 + (size_t)n * H * W * kC;
    const int cx = t >> 3, i = t & 7;           // decode: coarse column, fine row
    for (int x0 = 0; x0 < W; x0 += kTileCols) {
        // head on slot s = row r * HC + column c of the block, 32 slots per wave task
        for (int gi = wave; gi * 32 < NS; gi += 4) {
            const int s = gi * 32 + i32;
            const int r = s / HC, c = s % HC;
            const int yy = y0 + r - 1, xx = x0 + c - 1;
            const bool ok = s < NS && yy >= 0 && yy < H && xx >= 0 && xx < W;
            f32x16 acc[2];
            head_group<T>(act, ok ? (long)yy * W + xx : -1L, whs, bhs, acc);
            // row q of the 32 x 64 product belongs to slot gi * 32 + 8(q/4) + 4hk + q%4
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int s2 = gi * 32 + 8 * (q >> 2) + 4 * hk + (q & 3);
                if (s2 >= NS) continue;
                const int r2 = s2 / HC, c2 = s2 % HC;
                const int yq = y0 + r2 - 1, xq = x0 + c2 - 1;
                const bool okq = yq >= 0 && yq < H && xq >= 0 && xq < W;
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    const int k = nb * 32 + i32;
                    hs[r2][c2][k] = okq ? acc[nb][q] : -INFINITY;
                }
            }
        }
        __syncthreads();
        // decode the band's rows: thread t tests the 8 fine pixels (coarse column
        // t / 8, fine row t % 8) of each row, so thread order is the raster order
        // of the chunk within a row; a wave scan and the wave totals give every
        // candidate its slot
        const int x = x0 + cx;
        unsigned bits[kHdRows];
        int incl[kHdRows], cnt[kHdRows];
#pragma unroll
        for (int ry = 0; ry < kHdRows; ++ry) {
            bits[ry] = 0;
            if (x < W && y0 + ry < H) {
                float nv[3][kR + 2];
#pragma unroll
                for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                    for (int c = 0; c < kR + 2; ++c) {
                        const int fi = 7 + i + dz, fj = 7 + c;
                        nv[dz][c] = hs[ry + (fi >> 3)][cx + (fj >> 3)][(fi & 7) * kR + (fj & 7)];
                    }
#pragma unroll
                for (int j = 0; j < kR; ++j) {
                    const float v = nv[1][j + 1];
                    const bool cand = v >= thr && v > nv[0][j] && v > nv[0][j + 1] && v > nv[0][j + 2] &&
                                      v > nv[1][j] && v >= nv[1][j + 2] && v >= nv[2][j] &&
                                      v >= nv[2][j + 1] && v >= nv[2][j + 2];
                    bits[ry] |= cand ? 1u << j : 0u;
                }
            }
            cnt[ry] = __popc(bits[ry]);
            incl[ry] = cnt[ry];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(incl[ry], d);
                if (lane >= d) incl[ry] += v;
            }
            if (lane == 63) wave_tot[ry][wave] = incl[ry];
        }
        __syncthreads();
#pragma unroll
        for (int ry = 0; ry < kHdRows; ++ry) {
            if (!bits[ry]) continue;
            const int y = y0 + ry;
            int off = base_s[ry] + incl[ry] - cnt[ry];
            for (int q = 0; q < wave; ++q) off += wave_tot[ry][q];
            ulm_loc_t *out = staged + ((size_t)img * H + y) * row_cap;
            const float2 pv = P[((size_t)img * H + y) * W + x];
            const float inten = cnn_mag(pv);
            for (int j = 0; j < kR; ++j) {
                if (!(bits[ry] & (1u << j))) continue;
                if (off < row_cap) {
                    ulm_loc_t rec;
                    rec.plane = img / F;
                    rec.frame = img % F;
                    rec.iz = y;
                    rec.iu = x;
                    rec.z = ((float)(y * kR + i) + 0.5f) / kR - 0.5f;
                    rec.u = ((float)(x * kR + j) + 0.5f) / kR - 0.5f;
                    rec.ncc = hs[ry + 1][cx + 1][i * kR + j];
                    rec.intensity = inten;
                    out[off] = rec;
                }
                ++off;
            }
        }
        __syncthreads();       // hs and wave_tot are rewritten by the next chunk
        if (t < kHdRows) base_s[t] += wave_tot[t][0] + wave_tot[t][1] + wave_tot[t][2] + wave_tot[t][3];
        __syncthreads();
    }
    if (t < kHdRows && y0 + t < H) {
        row_cnt[(size_t)img * H + y0 + t] = min(base_s[t], row_cap);
        if (base_s[t] > row_cap) atomicOr(status, kStatusCnnRow);
    }
}

// ----------------------------------------------------------------- fused BF16 inference
// The whole BF16 inference of one horizontal strip of one image in one
// work-group: the input envelope, the six convolutions, the head and the
// decode run as a pipeline over the image columns, every stage one column of
// the strip per step, with each layer's recent columns held in LDS rings.  No
// activation reaches HBM; the only global traffic is the plane (read once) and
// the records.
//
// Strip: SH <= kFuseStrip decode rows ys .. ys + SH - 1.  A stage's column
// covers the rows its consumers need: layer j (j = 0 input, 1..6 conv0..conv5
// outputs, 7 heat) holds rows ys - e_j .. ys + SH + e_j - 1 with e = 7 - j for
// j <= 6 and e = 1 for the heat, so a 3x3 consumer reads producer indices
// c, c + 1, c + 2 for its index c.  Rows outside the image are stored as zero
// (the zero padding of every convolution), heat outside the image as -inf.
//
// Step it: stage j handles column it - lag_j, lags 0 (input), 2, 4, .., 12
// (conv0 .. conv5), 13 (head), 15 (decode).  A 3x3 consumer reads its
// producer's columns x - 1 .. x + 1, all written in earlier steps, so one
// barrier per step orders everything; 4-slot rings (2 for the head's input)
// are never overwritten while read.  Every stage also writes columns -1 and W
// (zeros; -inf for the heat), so the taps at the image's left and right edges
// read the zero padding from the rings like any other column.
//
// The arithmetic is the same as the layer-by-layer form (cnn_conv0_kernel,
// cnn_conv_kernel, cnn_head_decode_kernel): the same FMA order in conv0, the
// same MFMA sequence per output (taps in order, two channel-half chains summed
// at the end), the same epilogues and decode rule, so the records are
// identical.  The MFMAs run transposed (weights as the A operand, activations
// as B): each lane then ends with 16 channels of one pixel, written to LDS as
// four 8-byte runs.
//
// Waves (12): 0..9 conv1..conv5 (layer 1 + w/2, rows 32 (w & 1) ..), 0..6
// also the decode (8 lanes per row, one per fine row); 10..11 conv0 and the
// head, 11 also the input.  Activation slots hold 66 pixels x 32 channels, the
// 16-byte channel groups swizzled by (pixel / 2) mod 4 so 8 consecutive pixels
// read one group from 8 distinct bank groups.
constexpr int kFuseStrip = 50;                  // decode rows per strip at most
constexpr int kFuseSlot = 66;                   // pixels per activation slot
constexpr int kFuseHeatRows = kFuseStrip + 2;
constexpr int kFuseHeatStride = kR2 + 4;        // 16-byte aligned rows: the head writes float4
constexpr int kFuseInRows = kFuseStrip + 14;
constexpr int kFuseLagHead = 13, kFuseLagDecode = 15;
constexpr int kFuseThreads = 768;

__device__ inline int fuse_swz(int px) { return (px >> 1) & 3; }

__global__ __launch_bounds__(kFuseThreads, 1) void cnn_localize_fused_kernel(
    const float *__restrict__ p, const bf16 *__restrict__ wm, const float2 *__restrict__ P,
    const float *__restrict__ fmaxv, float thr, int H, int W, int F, int n_strips, int SH,
    ulm_loc_t *__restrict__ staged, int *__restrict__ row_cnt, int row_cap, int *__restrict__ status)
{
    __shared__ __attribute__((aligned(16))) bf16 ring[5][4][kFuseSlot * kC];    // conv0 .. conv4 outputs
    __shared__ __attribute__((aligned(16))) bf16 ring6[2][kFuseSlot * kC];      // conv5 output
    __shared__ float heat[4][kFuseHeatRows * kFuseHeatStride];
    __shared__ float x0r[4][kFuseInRows];
    __shared__ float inten[16][kFuseStrip];
    __shared__ float w0s[kW0 + kB0];
    __shared__ __attribute__((aligned(16))) bf16 whs[kR2 * Lds<bf16>::wh];
    __shared__ __attribute__((aligned(16))) float bhs[kR2];
    __shared__ __attribute__((aligned(16))) float bcs[kL - 1][kC];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i32 = lane & 31, hk = lane >> 5;
    const int img = blockIdx.x / n_strips, ys = (blockIdx.x % n_strips) * SH;
    for (int e = t; e < kW0 + kB0; e += kFuseThreads) w0s[e] = p[e];
    for (int e = t; e < (kL - 1) * kC; e += kFuseThreads) bcs[e / kC][e % kC] = p[off_b(1 + e / kC) + e % kC];
    stage_head<bf16>(p, whs, bhs);
    // heat rows of the strip outside the image hold -inf in every slot; the head
    // never writes them
    for (int e = t; e < 4 * kFuseHeatRows * kR2; e += kFuseThreads) {
        const int slot = e / (kFuseHeatRows * kR2), c = (e / kR2) % kFuseHeatRows, k = e % kR2;
        const int row = ys - 1 + c;
        if (row < 0 || row >= H) heat[slot][c * kFuseHeatStride + k] = -INFINITY;
    }
    const int n_it = W + kFuseLagDecode;

    // Two role loops, one barrier per step in each, so the conv weights held
    // by waves 0..9 are not live in the code of waves 10..11.
    if (wave < 10) {
        // ---- waves 0..9: conv1 .. conv5 (layer 1 + w/2, output rows 32 (w & 1) ..),
        // waves 0..6 also the decode
        const int layer = 1 + (wave >> 1), c0 = 32 * (wave & 1);
        bf16x8 wr[9][2];                             // A operand: output channel i32
        {
            const bf16 *wl = wm + (size_t)(layer - 1) * kWl + (size_t)i32 * 9 * kC;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    wr[tap][h] = *reinterpret_cast<const bf16x8 *>(wl + tap * kC + 16 * h + 8 * hk);
        }
        const bf16 *src = &ring[layer - 1][0][0];
        bf16 *dst0 = layer < 5 ? &ring[layer][0][0] : &ring6[0][0];
        const int dst_mask = layer < 5 ? 3 : 1, e_out = 6 - layer;
        const float *bl = bcs[layer - 1];
        // per-lane element offsets within a slot: the B operand of row offset dyy
        // and channel half h, and this lane's four output runs
        int loff[3][2], eoff[4];
#pragma unroll
        for (int dyy = 0; dyy < 3; ++dyy)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int pp = c0 + i32 + dyy;
                loff[dyy][h] = pp * kC + ((2 * h + hk) ^ fuse_swz(pp)) * 8;
            }
        const int c = c0 + i32;
#pragma unroll
        for (int r = 0; r < 4; ++r) eoff[r] = c * kC + (r ^ fuse_swz(c)) * 8 + 4 * hk;
        // decode lanes: row ys + (t >> 3), fine row t & 7; records of the row so far
        const int dy_rel = t >> 3, dfi = t & 7, dy = ys + dy_rel;
        const bool dec_ok = wave < 7 && dy_rel < SH && dy < H;
        int base = 0;
        // input lanes (wave 7): row ys - 7 + lane, the next two columns in flight
        const float m = fmaxv[img];
        const int in_row = ys - 7 + lane;
        const bool in_ok = wave == 7 && lane < SH + 14 && in_row >= 0 && in_row < H;
        const float2 *prow = P + ((size_t)img * H + (in_ok ? in_row : 0)) * W;
        auto in_load = [&](int x) { return in_ok && x < W ? prow[x] : make_float2(0.f, 0.f); };
        float2 pf0 = in_load(0), pf1 = in_load(1);
        __syncthreads();
        for (int it = -1; it < n_it; ++it) {
            // ---- input: x0 = |P| / frame max (0 outside the image), |P| kept for the
            // records; columns -1 and W are zero
            if (wave == 7 && it <= W) {
                float2 v = make_float2(0.f, 0.f);
                if (it >= 0 && it < W) {
                    v = pf0;
                    pf0 = pf1;
                    pf1 = in_load(it + 2);
                }
                if (lane < SH + 14) {
                    const float mag = cnn_mag(v);
                    x0r[it & 3][lane] = m > 0.f ? mag / m : 0.f;
                    if (lane >= 7 && lane < 7 + SH && it >= 0 && it < W) inten[it & 15][lane - 7] = mag;
                }
            }
            // columns -1 and W are written as zeros, so every read below is unconditional
            const int x = it - 2 * (layer + 1);
            if (x >= -1 && x <= W) {
                f32x16 a = {};
                if (x >= 0 && x < W) {
                    f32x16 acc[2] = {{}, {}};
                    // the next tap's operands are read while this tap's MFMAs run
                    int sb[3];
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) sb[dx] = ((x + dx - 1) & 3) * kFuseSlot * kC;
                    bf16x8 bv[2][2];
                    auto fetch = [&](int tap, int slot) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            bv[slot][h] = *reinterpret_cast<const bf16x8 *>(src + sb[tap % 3] + loff[tap / 3][h]);
                    };
                    fetch(0, 0);
#pragma unroll
                    for (int tap = 0; tap < 9; ++tap) {
                        if (tap + 1 < 9) fetch(tap + 1, (tap + 1) & 1);
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            acc[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[tap][h], bv[tap & 1][h], acc[h], 0,
                                                                            0, 0);
                    }
                    a = acc[0] + acc[1];
                }
                // lane holds output channels 8 (q / 4) + 4 hk + q % 4 of index c
                const int row = ys - e_out + c;
                const bool ok = x >= 0 && x < W && c < SH + 2 * e_out && row >= 0 && row < H;
                uint2 pk[4];                  // this lane's 16 channels, BF16, in 4 runs of 4
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float4 b4 = *reinterpret_cast<const float4 *>(&bl[8 * r + 4 * hk]);
                    const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
                    bf16 v4[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        v4[j] = fromf<bf16>(ok ? fmaxf(a[4 * r + j] + bb[j], 0.f) : 0.f);
                    pk[r] = *reinterpret_cast<const uint2 *>(v4);
                }
                bf16 *dst = dst0 + (x & dst_mask) * kFuseSlot * kC;
#pragma unroll
                for (int r = 0; r < 4; ++r) *reinterpret_cast<uint2 *>(dst + eoff[r]) = pk[r];
            }
            // ---- decode: 3x3 local maxima of the fine heatmap at or above thr,
            // records in (coarse column, fine row, fine column) order within each row
            const int xd = it - kFuseLagDecode;
            if (wave < 7 && xd >= 0 && xd < W) {
                // Lane t holds fine row 8 (t / 8) + t % 8 of the strip, so the fine
                // rows above and below a lane's are its neighbour lanes' own rows:
                // each lane reads its row (8 pixels of column xd and the edge pixel
                // of each neighbour column) and takes the other two by DPP wave
                // shifts; only the first and last lane of a wave read theirs.
                auto fine_row = [&](int dz, float (&r)[kR + 2]) {
                    const int fi = 7 + dfi + dz;
                    const int hrow = min(dy_rel + (fi >> 3), SH + 1);     // lanes past the strip: clamped
                    const float *hr = &heat[0][hrow * kFuseHeatStride + (fi & 7) * kR];
#pragma unroll
                    for (int cq = 0; cq < kR + 2; ++cq) {
                        const int fj = 7 + cq, col = xd - 1 + (fj >> 3);
                        r[cq] = hr[(col & 3) * kFuseHeatRows * kFuseHeatStride + (fj & 7)];
                    }
                };
                float r[kR + 2];
                fine_row(1, r);
                bool hot = false;
#pragma unroll
                for (int j = 0; j < kR; ++j) hot |= r[j + 1] >= thr;
                unsigned bits = 0;
                // with none of its pixels at or above thr (most of the heatmap) a
                // wave has no candidate and stops here
                if (__ballot(dec_ok && hot)) {
                    float r0[kR + 2], r2[kR + 2];
#pragma unroll
                    for (int cq = 0; cq < kR + 2; ++cq) {
                        const int x = __float_as_int(r[cq]);
                        r0[cq] = __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x138, 0xf, 0xf, false));  // wave_shr:1
                        r2[cq] = __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x130, 0xf, 0xf, false));  // wave_shl:1
                    }
                    if (lane == 0) fine_row(0, r0);
                    if (lane == 63) fine_row(2, r2);
                    if (dec_ok) {
                        // earlier neighbours in raster order must be below the pixel, later
                        // ones not above it: against the maxima of each side (the same
                        // decisions as the nine comparisons for finite heat values)
                        float p0[kR + 1], p2[kR + 1];
#pragma unroll
                        for (int j = 0; j <= kR; ++j) {
                            p0[j] = fmaxf(r0[j], r0[j + 1]);
                            p2[j] = fmaxf(r2[j], r2[j + 1]);
                        }
#pragma unroll
                        for (int j = 0; j < kR; ++j) {
                            const float v = r[j + 1];
                            const float before = fmaxf(fmaxf(p0[j], r0[j + 2]), r[j]);
                            const float after = fmaxf(fmaxf(p2[j], r2[j + 2]), r[j + 2]);
                            bits |= (v >= thr && v > before && v >= after) ? 1u << j : 0u;
                        }
                    }
                }
                // offsets within the row's 8 lanes (fine rows in order): an inclusive
                // scan by DPP row shifts, the row's total by quad swaps and the
                // half-row mirror (no LDS round trips)
                const int cnt = __popc(bits);
                int incl = cnt, u;
                u = __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, false);          // row_shr:1
                if (dfi >= 1) incl += u;
                u = __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, false);          // row_shr:2
                if (dfi >= 2) incl += u;
                u = __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, false);          // row_shr:4
                if (dfi >= 4) incl += u;
                int total = cnt;
                total += __builtin_amdgcn_update_dpp(0, total, 0xb1, 0xf, 0xf, false);     // quad_perm 1,0,3,2
                total += __builtin_amdgcn_update_dpp(0, total, 0x4e, 0xf, 0xf, false);     // quad_perm 2,3,0,1
                total += __builtin_amdgcn_update_dpp(0, total, 0x141, 0xf, 0xf, false);    // row_half_mirror
                if (bits) {
                    int off = base + incl - cnt;
                    ulm_loc_t *out = staged + ((size_t)img * H + dy) * row_cap;
                    const float iv = inten[xd & 15][dy_rel];
                    const float *hc = &heat[xd & 3][(dy_rel + 1) * kFuseHeatStride + dfi * kR];
                    for (int j = 0; j < kR; ++j) {
                        if (!(bits & (1u << j))) continue;
                        if (off < row_cap) {
                            ulm_loc_t rec;
                            rec.plane = img / F;
                            rec.frame = img % F;
                            rec.iz = dy;
                            rec.iu = xd;
                            rec.z = ((float)(dy * kR + dfi) + 0.5f) / kR - 0.5f;
                            rec.u = ((float)(xd * kR + j) + 0.5f) / kR - 0.5f;
                            rec.ncc = hc[j];
                            rec.intensity = iv;
                            out[off] = rec;
                        }
                        ++off;
                    }
                }
                base += total;
            }
            __syncthreads();
        }
        if (dec_ok && dfi == 0) {
            row_cnt[(size_t)img * H + dy] = min(base, row_cap);
            if (base > row_cap) atomicOr(status, kStatusCnnRow);
        }
    } else {
        // ---- waves 10..11: conv0 and the head
        const int tau = t - 640;                     // 0 .. 127
        const int c = 32 * (wave - 10) + i32;       // head: heat index of this lane
        float *const hrow0 = &heat[0][min(c, SH + 1) * kFuseHeatStride];
        const bool store = c < SH + 2, okh = store && ys - 1 + c >= 0 && ys - 1 + c < H;
        __syncthreads();
        // conv0 items of this thread all have channel group tau & 3: its 8
        // channels' weights and biases stay in registers
        const int cc = tau & 3;
        float w0r[8][9], b0r[8];
#pragma unroll
        for (int o8 = 0; o8 < 8; ++o8) {
#pragma unroll
            for (int k = 0; k < 9; ++k) w0r[o8][k] = w0s[(8 * cc + o8) * 9 + k];
            b0r[o8] = w0s[kW0 + 8 * cc + o8];
        }
        for (int it = -1; it < n_it; ++it) {
            // ---- conv0 (1 -> 32): item = (output index, 8-channel group)
            const int x = it - 2;
            if (x >= -1 && x <= W) {
                const bool col_ok = x >= 0 && x < W;
                for (int item = tau; item < (SH + 12) * 4; item += 128) {
                    const int pi = item >> 2;
                    const int row = ys - 6 + pi;
                    const bool ok = col_ok && row >= 0 && row < H;
                    bf16 res[8] = {};
                    if (col_ok) {
                        float in[9];
#pragma unroll
                        for (int dyy = 0; dyy < 3; ++dyy)
#pragma unroll
                            for (int dx = 0; dx < 3; ++dx) in[dyy * 3 + dx] = x0r[(x + dx - 1) & 3][pi + dyy];
#pragma unroll
                        for (int o8 = 0; o8 < 8; ++o8) {
                            float s = 0.f;
#pragma unroll
                            for (int k = 0; k < 9; ++k) s = fmaf(w0r[o8][k], in[k], s);
                            res[o8] = fromf<bf16>(ok ? fmaxf(s + b0r[o8], 0.f) : 0.f);
                        }
                    }
                    *reinterpret_cast<uint4 *>(&ring[0][x & 3][(pi * 4 + (cc ^ fuse_swz(pi))) * 8]) =
                        *reinterpret_cast<const uint4 *>(res);
                }
            }
            // ---- head (1x1, 32 -> 64) on conv5's column: 32 rows x 64 outputs per
            // wave, the MFMAs started from the bias; rows outside the image keep
            // the -inf written at the start, columns -1 and W are all -inf
            const int xh = it - kFuseLagHead;
            float *hrow = hrow0 + (xh & 3) * kFuseHeatRows * kFuseHeatStride;
            if ((xh == -1 || xh == W) && store) {
                const float4 ninf = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
#pragma unroll
                for (int k = 0; k < kR2; k += 4) *reinterpret_cast<float4 *>(&hrow[k]) = ninf;
            }
            if (xh >= 0 && xh < W) {
                f32x16 hacc[2];
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float4 b4 = *reinterpret_cast<const float4 *>(&bhs[nb * 32 + 8 * r + 4 * hk]);
                        hacc[nb][4 * r + 0] = b4.x;
                        hacc[nb][4 * r + 1] = b4.y;
                        hacc[nb][4 * r + 2] = b4.z;
                        hacc[nb][4 * r + 3] = b4.w;
                    }
                const bf16 *pix = &ring6[xh & 1][c * kC];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(pix + ((2 * h + hk) ^ fuse_swz(c)) * 8);
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) {
                        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(
                            whs + (nb * 32 + i32) * Lds<bf16>::wh + h * 16 + hk * 8);
                        hacc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, hacc[nb], 0, 0, 0);
                    }
                }
                if (okh) {
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            *reinterpret_cast<float4 *>(&hrow[nb * 32 + 8 * r + 4 * hk]) =
                                make_float4(hacc[nb][4 * r], hacc[nb][4 * r + 1], hacc[nb][4 * r + 2],
                                            hacc[nb][4 * r + 3]);
                }
            }
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------- training
// target T[n][y][x][k] (the logits layout), float bits: max over MBs of the blob
__global__ void cnn_target_kernel(const float2 *__restrict__ mb, const int *__restrict__ mb_img,
                                  int n_mb, int B, int *__restrict__ T, int H, int W)
{
    const int m = blockIdx.x;
    if (m >= n_mb) return;
    const int n = mb_img[m];
    if (n < 0 || n >= B) return;
    const float2 zu = mb[m];
    if (!(fabsf(zu.x) < 1e6f && fabsf(zu.y) < 1e6f)) return;
    const float cz = kR * (zu.x + 0.5f) - 0.5f, cu = kR * (zu.y + 0.5f) - 0.5f;
    constexpr int rad = 4, side = 2 * rad + 2;
    const int fz0 = (int)floorf(cz) - rad, fu0 = (int)floorf(cu) - rad;
    for (int e = threadIdx.x; e < side * side; e += blockDim.x) {
        const int fz = fz0 + e / side, fu = fu0 + e % side;
        if (fz < 0 || fu < 0 || fz >= H * kR || fu >= W * kR) continue;
        const float dz = fz - cz, du = fu - cu;
        const float g = expf(-(dz * dz + du * du) * 0.5f);
        const int y = fz / kR, i = fz % kR, x = fu / kR, j = fu % kR;
        atomicMax(&T[(((size_t)n * H + y) * W + x) * kR2 + i * kR + j], __float_as_int(g));
    }
}

// per-block loss partial sums and the logit gradient g = 2 (h - T) / count
__global__ __launch_bounds__(256) void cnn_loss_kernel(const float *__restrict__ logits,
                                                       const int *__restrict__ T,
                                                       float *__restrict__ g, size_t count,
                                                       double *__restrict__ part)
{
    double s = 0.0;
    const double scale = 2.0 / (double)count;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x) {
        const float d = logits[i] - __int_as_float(T[i]);
        s += (double)d * d;
        g[i] = (float)(scale * d);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void cnn_loss_final_kernel(const double *__restrict__ part, int n, double inv_count,
                                      float *__restrict__ loss)
{
    __shared__ double red[64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int i = 0; i < 64; ++i) tot += red[i];
        *loss = (float)(tot * inv_count);
    }
}

// head backward, per pixel: dz6[c] = (sum_k wh[k][c] g[k]) where a6[c] > 0, else 0
template <typename T>
__global__ __launch_bounds__(256) void cnn_head_bwd_data_kernel(const float *__restrict__ g,
                                                                const float *__restrict__ p,
                                                                const T *__restrict__ a6,
                                                                T *__restrict__ dz6, size_t npx)
{
    __shared__ float wh[kR2][kC];
    for (int e = threadIdx.x; e < kR2 * kC; e += blockDim.x) wh[e / kC][e % kC] = p[off_wh() + e];
    __syncthreads();
    const size_t px = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (px >= npx) return;
    float acc[kC];
#pragma unroll
    for (int c = 0; c < kC; ++c) acc[c] = 0.f;
    const float4 *gs = reinterpret_cast<const float4 *>(g + px * kR2);
    for (int k4 = 0; k4 < kR2 / 4; ++k4) {
        const float4 v = gs[k4];
        const float gv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < kC; ++c) acc[c] = fmaf(wh[k4 * 4 + i][c], gv[i], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kC; ++c) {
        const bool on = tof(a6[px * kC + c]) > 0.f;
        dz6[px * kC + c] = fromf<T>(on ? acc[c] : 0.f);
    }
}

// Head weight-gradient partials.  Work-group w takes the 128-pixel chunks
// w, w + G, ...; thread t owns (k, c) = ((t + 256 m) / 32, t % 32), m < 8, and
// the bias k = t for t < 64.  part[w][k][c] then part[w][2048 + k].
template <typename T>
__global__ __launch_bounds__(256) void cnn_head_bwd_weight_kernel(const float *__restrict__ g,
                                                                  const T *__restrict__ a6,
                                                                  float *__restrict__ part, size_t npx)
{
    __shared__ float gs[kHeadPx][kR2 + 1];
    __shared__ float as[kHeadPx][kC + 1];
    const int t = threadIdx.x;
    float acc[8] = {}, accb = 0.f;
    const size_t nchunks = (npx + kHeadPx - 1) / kHeadPx;
    for (size_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const size_t p0 = ch * kHeadPx;
        const int np = (int)std::min((size_t)kHeadPx, npx - p0);
        __syncthreads();
        for (int e = t; e < kHeadPx * kR2; e += 256) {
            const int r = e / kR2, k = e % kR2;
            gs[r][k] = r < np ? g[(p0 + r) * kR2 + k] : 0.f;
        }
        for (int e = t; e < kHeadPx * kC; e += 256) {
            const int r = e / kC, c = e % kC;
            as[r][c] = r < np ? tof(a6[(p0 + r) * kC + c]) : 0.f;
        }
        __syncthreads();
        const int c = t % kC;
        for (int r = 0; r < np; ++r) {
            const float a = as[r][c];
#pragma unroll
            for (int m = 0; m < 8; ++m) acc[m] = fmaf(gs[r][(t + 256 * m) / kC], a, acc[m]);
            if (t < kR2) accb += gs[r][t];
        }
    }
    float *dst = part + (size_t)blockIdx.x * (kWh + kBh);
#pragma unroll
    for (int m = 0; m < 8; ++m) dst[t + 256 * m] = acc[m];
    if (t < kR2) dst[kWh + t] = accb;
}

// Conv weight-gradient partials (layers 1..5).  Work-group w takes tiles
// w, w + G, ... of 4 x 32 pixels; thread t owns the pairs (o, c) =
// ((t + 256 m) / 32, t % 32), m < 4, for all 9 taps, and the bias o = t for t < 32.
// part[w][o][c][tap] then part[w][9216 + o].
template <typename T>
__global__ __launch_bounds__(256) void cnn_conv_bwd_weight_kernel(const T *__restrict__ x,
                                                                  const T *__restrict__ dz,
                                                                  float *__restrict__ part, int H,
                                                                  int W, int B)
{
    constexpr int TC = kTileCols + 2;
    __shared__ float xs[kTileRows + 2][TC][kC + 1];
    __shared__ float ds[kTileRows][kTileCols][kC + 1];
    const int t = threadIdx.x, c = t % kC;
    const int tx = cdiv(W, kTileCols), ty = cdiv(H, kTileRows);
    const long ntiles = (long)tx * ty * B;
    float acc[4][9] = {};
    float accb = 0.f;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int n = tile / ((long)tx * ty), y0 = (tile / tx) % ty * kTileRows,
                  x0 = tile % tx * kTileCols;
        __syncthreads();
        for (int e = t; e < (kTileRows + 2) * TC * kC; e += 256) {
            const int cc = e % kC, px = (e / kC) % TC, ry = e / (kC * TC);
            const int yy = y0 + ry - 1, xx = x0 + px - 1;
            xs[ry][px][cc] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                                 ? tof(x[(((size_t)n * H + yy) * W + xx) * kC + cc]) : 0.f;
        }
        for (int e = t; e < kTileRows * kTileCols * kC; e += 256) {
            const int cc = e % kC, px = (e / kC) % kTileCols, ry = e / (kC * kTileCols);
            const int yy = y0 + ry, xx = x0 + px;
            ds[ry][px][cc] = (yy < H && xx < W) ? tof(dz[(((size_t)n * H + yy) * W + xx) * kC + cc]) : 0.f;
        }
        __syncthreads();
        for (int ry = 0; ry < kTileRows; ++ry)
            for (int px = 0; px < kTileCols; ++px) {
                float xv[9];
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) xv[tap] = xs[ry + tap / 3][px + tap % 3][c];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float d = ds[ry][px][(t + 256 * m) / kC];
#pragma unroll
                    for (int tap = 0; tap < 9; ++tap) acc[m][tap] = fmaf(d, xv[tap], acc[m][tap]);
                }
                if (t < kC) accb += ds[ry][px][t];
            }
    }
    float *dst = part + (size_t)blockIdx.x * (kWl + kBl);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int o = (t + 256 * m) / kC;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) dst[(o * kC + c) * 9 + tap] = acc[m][tap];
    }
    if (t < kC) dst[kWl + t] = accb;
}

// Layer-0 weight-gradient partials: thread t < 288 owns (o, tap) = (t / 9, t % 9),
// 288 <= t < 320 the bias o = t - 288.  part[w][o][tap] then part[w][288 + o].
template <typename T>
__global__ __launch_bounds__(320) void cnn_conv0_bwd_weight_kernel(const float *__restrict__ x0,
                                                                   const T *__restrict__ dz,
                                                                   float *__restrict__ part, int H,
                                                                   int W, int B)
{
    constexpr int TC = kTileCols + 2;
    __shared__ float xs[kTileRows + 2][TC];
    __shared__ float ds[kTileRows][kTileCols][kC + 1];
    const int t = threadIdx.x;
    const int tx = cdiv(W, kTileCols), ty = cdiv(H, kTileRows);
    const long ntiles = (long)tx * ty * B;
    const int o = t < kW0 ? t / 9 : t - kW0, tap = t < kW0 ? t % 9 : 4;
    const int dy = tap / 3, dx = tap % 3;
    float acc = 0.f;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int n = tile / ((long)tx * ty), y0 = (tile / tx) % ty * kTileRows,
                  x0c = tile % tx * kTileCols;
        __syncthreads();
        for (int e = t; e < (kTileRows + 2) * TC; e += blockDim.x) {
            const int px = e % TC, ry = e / TC;
            const int yy = y0 + ry - 1, xx = x0c + px - 1;
            xs[ry][px] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? x0[((size_t)n * H + yy) * W + xx] : 0.f;
        }
        for (int e = t; e < kTileRows * kTileCols * kC; e += blockDim.x) {
            const int cc = e % kC, px = (e / kC) % kTileCols, ry = e / (kC * kTileCols);
            const int yy = y0 + ry, xx = x0c + px;
            ds[ry][px][cc] = (yy < H && xx < W) ? tof(dz[(((size_t)n * H + yy) * W + xx) * kC + cc]) : 0.f;
        }
        __syncthreads();
        for (int ry = 0; ry < kTileRows; ++ry)
            for (int px = 0; px < kTileCols; ++px)
                acc = t < kW0 ? fmaf(ds[ry][px][o], xs[ry + dy][px + dx], acc) : acc + ds[ry][px][o];
    }
    part[(size_t)blockIdx.x * (kW0 + kB0) + t] = acc;
}

// grad[off + e] = sum over the partials q of part[q][e] (FP64, fixed order)
__global__ void cnn_reduce_kernel(const float *__restrict__ part, int nparts, int width,
                                  float *__restrict__ grad, int off)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= width) return;
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += part[(size_t)q * width + e];
    grad[off + e] = (float)s;
}

__global__ void cnn_adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                const float *__restrict__ g, int n, float lr, float b1, float b2,
                                float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------------- host side
static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace regions for a batch of B images of H x W pixels.
struct CnnLayout {
    size_t x0, act[kL], dz[2], logits, target, glog, wm, wt, part, lpart, grad, total;
    int n_act;
};
constexpr int kLossParts = 1024;

static CnnLayout cnn_layout(int B, int H, int W, bool fp32, bool train) {
    const size_t npx = (size_t)B * H * W, es = fp32 ? 4 : 2;
    CnnLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += a256(bytes); return at; };
    L.x0 = take(sizeof(float) * npx);
    L.n_act = train ? kL : 2;
    for (int l = 0; l < L.n_act; ++l) L.act[l] = take(es * npx * kC);
    L.wm = take(es * (kL - 1) * kWl);
    L.wt = take(es * (kL - 1) * kWl);
    L.logits = take(sizeof(float) * npx * kR2);
    if (train) {
        L.dz[0] = take(es * npx * kC);
        L.dz[1] = take(es * npx * kC);
        L.target = take(sizeof(float) * npx * kR2);
        L.glog = take(sizeof(float) * npx * kR2);
        L.part = take(sizeof(float) * kMaxPartials * (kWl + kBl));
        L.lpart = take(sizeof(double) * kLossParts);
        L.grad = take(sizeof(float) * kParams);
    }
    L.total = o;
    return L;
}

size_t cnn_workspace_bytes(int B, int H, int W, bool fp32, bool train) {
    return cnn_layout(B, H, W, fp32, train).total;
}

// Localisation workspace: the batch buffers (no logits) plus the per-row staging.
struct CnnLocLayout { size_t x0, act[2], wm, wt, staged, cnt, off, total; int row_cap; };

static CnnLocLayout cnn_loc_layout(int batch, int H, int W, int n_img, bool fp32) {
    const size_t npx = (size_t)batch * H * W, es = fp32 ? 4 : 2;
    CnnLocLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += a256(bytes); return at; };
    L.row_cap = std::max(16, cdiv(W, 2));
    L.x0 = take(sizeof(float) * npx);
    L.act[0] = take(es * npx * kC);
    L.act[1] = take(es * npx * kC);
    L.wm = take(es * (kL - 1) * kWl);
    L.wt = take(es * (kL - 1) * kWl);
    L.staged = take(sizeof(ulm_loc_t) * (size_t)n_img * H * L.row_cap);
    L.cnt = take(sizeof(int) * (size_t)n_img * H);
    L.off = take(sizeof(int) * (size_t)n_img * H);
    L.total = o;
    return L;
}

size_t cnn_loc_workspace_bytes(int batch, int H, int W, int n_img, bool fp32) {
    return cnn_loc_layout(batch, H, W, n_img, fp32).total;
}

// Persistent conv grid: enough work-groups to fill every CU a few times over.
static unsigned conv_grid(int B, int H, int W) {
    const long tiles = (long)cdiv(W, kTileCols) * cdiv(H, kTileRows) * B;
    return (unsigned)std::min(tiles, 256L * 8);
}

static unsigned conv_fwd_grid(int B, int H, int W) {
    const long tiles = (long)cdiv(W, kTileCols) * cdiv(H, kCvRows) * B;
    return (unsigned)std::min(tiles, 256L * 4);
}

template <typename T>
static hipError_t run_forward(const float *params, const float *x0, T *const *act, int n_act,
                              T *wm, T *wt, int B, int H, int W, hipStream_t st, int *last)
{
    const size_t npx = (size_t)B * H * W;
    hipLaunchKernelGGL(cnn_prepare_kernel<T>, dim3(cdiv((kL - 1) * kWl, 256)), dim3(256), 0, st,
                       params, wm, wt);
    hipLaunchKernelGGL(cnn_conv0_kernel<T>, dim3((unsigned)cdiv(npx, (size_t)256)), dim3(256), 0, st,
                       x0, params, act[0], H, W, npx);
    const dim3 grid(conv_grid(B, H, W));
    int cur = 0;
    for (int l = 1; l < kL; ++l) {
        const int nxt = n_act == kL ? l : cur ^ 1;
        if constexpr (sizeof(T) == 2)
            hipLaunchKernelGGL(cnn_conv_fwd_bf16_kernel, dim3(conv_fwd_grid(B, H, W)), dim3(256), 0, st,
                               act[cur], wm + (size_t)(l - 1) * kWl, params + off_b(l), act[nxt], H, W,
                               B);
        else
            hipLaunchKernelGGL((cnn_conv_kernel<T, false>), grid, dim3(256), 0, st, act[cur],
                               wm + (size_t)(l - 1) * kWl, params + off_b(l), (const T *)nullptr,
                               act[nxt], H, W, B);
        cur = nxt;
    }
    *last = cur;
    return hipGetLastError();
}

template <typename T>
static hipError_t forward_heat_t(const float *params, const float *x0, float *heat, int B, int H,
                                 int W, char *ws, hipStream_t st)
{
    const CnnLayout L = cnn_layout(B, H, W, sizeof(T) == 4, false);
    T *act[2] = {(T *)(ws + L.act[0]), (T *)(ws + L.act[1])};
    int last = 0;
    hipError_t e = run_forward<T>(params, x0, act, 2, (T *)(ws + L.wm), (T *)(ws + L.wt), B, H, W,
                                  st, &last);
    if (e != hipSuccess) return e;
    const size_t npx = (size_t)B * H * W;
    float *logits = (float *)(ws + L.logits);
    hipLaunchKernelGGL(cnn_head_kernel<T>, dim3((unsigned)cdiv(npx, (size_t)128)), dim3(256), 0, st,
                       act[last], params, logits, npx);
    const size_t total = npx * kR2;
    hipLaunchKernelGGL(cnn_d2s_kernel, dim3((unsigned)cdiv(total, (size_t)256)), dim3(256), 0, st,
                       logits, heat, H, W, total);
    return hipGetLastError();
}

hipError_t cnn_forward_heat(const float *params, const float *x0, float *heat, int B, int H, int W,
                            bool fp32, char *ws, hipStream_t st)
{
    return fp32 ? forward_heat_t<float>(params, x0, heat, B, H, W, ws, st)
                : forward_heat_t<bf16>(params, x0, heat, B, H, W, ws, st);
}

template <typename T>
static hipError_t gradients_t(const float *params, const float *x0, const float *mb_zu,
                              const int *mb_img, int n_mb, int B, int H, int W, float *grad,
                              float *loss, char *ws, hipStream_t st)
{
    const CnnLayout L = cnn_layout(B, H, W, sizeof(T) == 4, true);
    T *act[kL];
    for (int l = 0; l < kL; ++l) act[l] = (T *)(ws + L.act[l]);
    T *dz[2] = {(T *)(ws + L.dz[0]), (T *)(ws + L.dz[1])};
    float *logits = (float *)(ws + L.logits), *glog = (float *)(ws + L.glog);
    int *target = (int *)(ws + L.target);
    float *part = (float *)(ws + L.part);
    double *lpart = (double *)(ws + L.lpart);
    const size_t npx = (size_t)B * H * W, count = npx * kR2;
    int last = 0;
    hipError_t e = run_forward<T>(params, x0, act, kL, (T *)(ws + L.wm), (T *)(ws + L.wt), B, H, W,
                                  st, &last);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cnn_head_kernel<T>, dim3((unsigned)cdiv(npx, (size_t)128)), dim3(256), 0, st,
                       act[kL - 1], params, logits, npx);
    // target and loss
    hipLaunchKernelGGL(cnn_fill_kernel, dim3(1024), dim3(256), 0, st, target, count, 0);
    if (n_mb > 0)
        hipLaunchKernelGGL(cnn_target_kernel, dim3(n_mb), dim3(128), 0, st, (const float2 *)mb_zu,
                           mb_img, n_mb, B, target, H, W);
    hipLaunchKernelGGL(cnn_loss_kernel, dim3(kLossParts), dim3(256), 0, st, logits, target, glog,
                       count, lpart);
    hipLaunchKernelGGL(cnn_loss_final_kernel, dim3(1), dim3(64), 0, st, lpart, kLossParts,
                       1.0 / (double)count, loss);
    // head
    const int gh = (int)std::min((size_t)kMaxPartials, cdiv(npx, (size_t)kHeadPx));
    hipLaunchKernelGGL(cnn_head_bwd_weight_kernel<T>, dim3(gh), dim3(256), 0, st, glog, act[kL - 1],
                       part, npx);
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3(cdiv(kWh + kBh, 256)), dim3(256), 0, st, part, gh,
                       kWh + kBh, grad, off_wh());
    hipLaunchKernelGGL(cnn_head_bwd_data_kernel<T>, dim3((unsigned)cdiv(npx, (size_t)256)), dim3(256),
                       0, st, glog, params, act[kL - 1], dz[0], npx);
    // conv layers 5..1: weight gradient, then the data gradient through the mask below
    const dim3 grid(cdiv(W, kTileCols), cdiv(H, kTileRows), B);
    const long ntiles = (long)grid.x * grid.y * grid.z;
    const int gw = (int)std::min((long)kMaxPartials, ntiles);
    const T *wt = (const T *)(ws + L.wt);
    int cur = 0;
    for (int l = kL - 1; l >= 1; --l) {
        hipLaunchKernelGGL(cnn_conv_bwd_weight_kernel<T>, dim3(gw), dim3(256), 0, st, act[l - 1],
                           dz[cur], part, H, W, B);
        hipLaunchKernelGGL(cnn_reduce_kernel, dim3(cdiv(kWl + kBl, 256)), dim3(256), 0, st, part, gw,
                           kWl + kBl, grad, off_w(l));
        hipLaunchKernelGGL((cnn_conv_kernel<T, true>), dim3(conv_grid(B, H, W)), dim3(256), 0, st,
                           dz[cur], wt + (size_t)(l - 1) * kWl, (const float *)nullptr,
                           act[l - 1], dz[cur ^ 1], H, W, B);
        cur ^= 1;
    }
    hipLaunchKernelGGL(cnn_conv0_bwd_weight_kernel<T>, dim3(gw), dim3(kW0 + kB0), 0, st, x0, dz[cur],
                       part, H, W, B);
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3(cdiv(kW0 + kB0, 256)), dim3(256), 0, st, part, gw,
                       kW0 + kB0, grad, 0);
    return hipGetLastError();
}

hipError_t cnn_gradients(const float *params, const float *x0, const float *mb_zu,
                         const int *mb_img, int n_mb, int B, int H, int W, bool fp32, float *grad,
                         float *loss, char *ws, hipStream_t st)
{
    return fp32 ? gradients_t<float>(params, x0, mb_zu, mb_img, n_mb, B, H, W, grad, loss, ws, st)
                : gradients_t<bf16>(params, x0, mb_zu, mb_img, n_mb, B, H, W, grad, loss, ws, st);
}

float *cnn_ws_grad(int B, int H, int W, bool fp32, char *ws) {
    return (float *)(ws + cnn_layout(B, H, W, fp32, true).grad);
}

hipError_t cnn_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                    hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - pow((double)b1, step)), c2 = (float)(1.0 - pow((double)b2, step));
    hipLaunchKernelGGL(cnn_adam_kernel, dim3(cdiv(kParams, 256)), dim3(256), 0, st, params, m, v,
                       grad, kParams, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t cnn_images(const float2 *P, const float *fmax, float *x0, int npix, int n0, int nb,
                      hipStream_t st)
{
    hipLaunchKernelGGL(cnn_input_kernel, dim3(cdiv(npix, 256), nb), dim3(256), 0, st, P, fmax, x0,
                       npix, n0);
    return hipGetLastError();
}

hipError_t launch_compact(const int *cnt, int *off, int nslots, int *count, const ulm_loc_t *staged,
                          int cap, ulm_loc_t *locs, int capacity, hipStream_t st);

template <typename T>
static hipError_t localize_t(const float *params, const float2 *P, const float *fmax, float thr,
                             int n_img, int F, int H, int W, int batch, ulm_loc_t *locs,
                             int capacity, int *count, int *status, char *cws, hipStream_t st)
{
    const CnnLocLayout L = cnn_loc_layout(batch, H, W, n_img, sizeof(T) == 4);
    float *x0 = (float *)(cws + L.x0);
    T *act[2] = {(T *)(cws + L.act[0]), (T *)(cws + L.act[1])};
    ulm_loc_t *staged = (ulm_loc_t *)(cws + L.staged);
    int *cnt = (int *)(cws + L.cnt), *off = (int *)(cws + L.off);
    hipLaunchKernelGGL(cnn_status_clear_kernel, dim3(1), dim3(64), 0, st, status, kStatusCnnRow);
    if constexpr (sizeof(T) == 2) {
        // BF16: the fused strip pipeline over every image at once
        hipLaunchKernelGGL(cnn_prepare_kernel<T>, dim3(cdiv((kL - 1) * kWl, 256)), dim3(256), 0, st,
                           params, (T *)(cws + L.wm), (T *)(cws + L.wt));
        const int n_strips = cdiv(H, kFuseStrip), SH = cdiv(H, n_strips);
        hipLaunchKernelGGL(cnn_localize_fused_kernel, dim3((unsigned)((long)n_img * n_strips)),
                           dim3(kFuseThreads), 0, st, params, (const bf16 *)(cws + L.wm), P, fmax, thr,
                           H, W, F, n_strips, SH, staged, cnt, L.row_cap, status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_compact(cnt, off, n_img * H, count, staged, L.row_cap, locs, capacity, st);
    } else {
        // FP32: layer by layer, `batch` images per pass, head and decode fused
        for (int n0 = 0; n0 < n_img; n0 += batch) {
            const int nb = std::min(batch, n_img - n0);
            hipError_t e = cnn_images(P, fmax, x0, H * W, n0, nb, st);
            if (e != hipSuccess) return e;
            int last = 0;
            if ((e = run_forward<T>(params, x0, act, 2, (T *)(cws + L.wm), (T *)(cws + L.wt), nb, H, W,
                                    st, &last)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(cnn_head_decode_kernel<T>, dim3(cdiv(H, kHdRows), nb), dim3(256), 0, st,
                               act[last], params, P, thr, H, W, n0, F, staged, cnt, L.row_cap, status);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        return launch_compact(cnt, off, n_img * H, count, staged, L.row_cap, locs, capacity, st);
    }
}

hipError_t cnn_localize(const float *params, const float2 *P, const float *fmax, float thr,
                        int n_img, int F, int H, int W, int batch, bool fp32, ulm_loc_t *locs,
                        int capacity, int *count, int *status, char *cws, hipStream_t st)
{
    return fp32 ? localize_t<float>(params, P, fmax, thr, n_img, F, H, W, batch, locs, capacity,
                                    count, status, cws, st)
                : localize_t<bf16>(params, P, fmax, thr, n_img, F, H, W, batch, locs, capacity,
                                   count, status, cws, st);
}

}  // namespace ulm
