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
    x0[(size_t)n * npix + i] = m > 0.f ? sqrtf(v.x * v.x + v.y * v.y) / m : 0.f;
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

// ----------------------------------------------------------------- head
// Stage the head weights (T, padded rows) and biases in LDS.
template <typename T>
__device__ inline void stage_head(const float *__restrict__ p, T *whs, float *bhs) {
    constexpr int WS = Lds<T>::wh;
    for (int e = threadIdx.x; e < kWh; e += blockDim.x) whs[(e / kC) * WS + e % kC] = fromf<T>(p[off_wh() + e]);
    for (int e = threadIdx.x; e < kBh; e += blockDim.x) bhs[e] = p[off_bh() + e];
}

// One wave: 32 pixels (lane i32 supplies pixel `px`, or none when px < 0) x 64
// head outputs.  acc[nb][q] = sum_c wh[32 nb + i32][c] a[pixel 8(q/4) + 4hk + q%4][c]
template <typename T>
__device__ inline void head_group(const T *__restrict__ act, long px, const T *whs, f32x16 acc[2]) {
    constexpr int WS = Lds<T>::wh;
    const int lane = threadIdx.x & 63, i32 = lane & 31, hk = lane >> 5;
    acc[0] = f32x16{};
    acc[1] = f32x16{};
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

// logits[px][k] = bh[k] + sum_c wh[k][c] a6[px][c]; 32 pixels per wave
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
    head_group<T>(a6, mine, whs, acc);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const size_t px = base + 8 * (q >> 2) + 4 * hk + (q & 3);
            const int k = nb * 32 + i32;
            if (px < npx) logits[px * kR2 + k] = acc[nb][q] + bhs[k];
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
// One work-group per (image, coarse row y).  For each 32-column chunk the head
// runs on coarse rows y-1, y, y+1 and columns x0-1 .. x0+32 (waves 0-2: the
// three rows, wave 3: the six edge pixels), giving every fine pixel of row y its
// 8 fine neighbours.  Candidates: heat >= thr, heat above the neighbours earlier
// in fine raster order and not below the later ones.  Records are compacted in
// (coarse column, fine row, fine column) order into the row's staging slot.
template <typename T>
__global__ __launch_bounds__(256, 4) void cnn_head_decode_kernel(
    const T *__restrict__ a6, const float *__restrict__ p, const float2 *__restrict__ P, float thr,
    int H, int W, int n0, int F, ulm_loc_t *__restrict__ staged, int *__restrict__ row_cnt,
    int row_cap, int *__restrict__ status)
{
    constexpr int HC = kTileCols + 2;
    __shared__ __attribute__((aligned(16))) T whs[kR2 * Lds<T>::wh];
    __shared__ float bhs[kR2];
    __shared__ float hs[3][HC][kR2 + 1];       // +1: the decode's 64 lanes (8 columns x 8 fine rows) hit 64 banks
    __shared__ int wave_tot[4];
    __shared__ int base_s;
    stage_head<T>(p, whs, bhs);
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const int y = blockIdx.x, n = blockIdx.y, img = n0 + n;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i32 = lane & 31, hk = lane >> 5;
    const T *act = a6 + (size_t)n * H * W * kC;
    ulm_loc_t *out = staged + ((size_t)img * H + y) * row_cap;
    for (int x0 = 0; x0 < W; x0 += kTileCols) {
        // the pixel this lane supplies: row r (0..2 = y-1..y+1), chunk column cc (0..33)
        int r, cc;
        if (wave < 3) { r = wave; cc = 1 + i32; }
        else if (i32 < 6) { r = i32 >> 1; cc = (i32 & 1) ? HC - 1 : 0; }
        else { r = -1; cc = 0; }
        const int yy = y + r - 1, xx = x0 + cc - 1;
        const bool ok = r >= 0 && yy >= 0 && yy < H && xx >= 0 && xx < W;
        f32x16 acc[2];
        head_group<T>(act, ok ? (long)yy * W + xx : -1L, whs, acc);
        // row q of the 32 x 64 product belongs to the pixel of lane 8(q/4) + 4hk + q%4
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int src = 8 * (q >> 2) + 4 * hk + (q & 3);
            if (wave == 3 && src >= 6) continue;
            const int rr = wave < 3 ? wave : src >> 1;
            const int c2 = wave < 3 ? 1 + src : ((src & 1) ? HC - 1 : 0);
            const int yq = y + rr - 1, xq = x0 + c2 - 1;
            const bool okq = yq >= 0 && yq < H && xq >= 0 && xq < W;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int k = nb * 32 + i32;
                hs[rr][c2][k] = okq ? acc[nb][q] + bhs[k] : -INFINITY;
            }
        }
        __syncthreads();
        // decode the 32 x 64 fine pixels of row y in this chunk: thread t tests the
        // 8 fine pixels (coarse column t / 8, fine row t % 8), so thread order is
        // the raster order of the chunk; a wave scan and the wave totals give
        // every candidate its slot
        const int cx = t >> 3, i = t & 7, x = x0 + cx;
        unsigned bits = 0;
        float vals[kR];
        if (x < W) {
            // fine rows i-1..i+1 and fine columns -1..8 around this thread's 8 pixels,
            // read once (fine offsets are taken within coarse rows y-1..y+1 and
            // columns x-1..x+1 of the chunk)
            float nv[3][kR + 2];
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int c = 0; c < kR + 2; ++c) {
                    const int fi = 7 + i + dz, fj = 7 + c;
                    nv[dz][c] = hs[fi >> 3][cx + (fj >> 3)][(fi & 7) * kR + (fj & 7)];
                }
#pragma unroll
            for (int j = 0; j < kR; ++j) {
                const float v = nv[1][j + 1];
                vals[j] = v;
                const bool cand = v >= thr && v > nv[0][j] && v > nv[0][j + 1] && v > nv[0][j + 2] &&
                                  v > nv[1][j] && v >= nv[1][j + 2] && v >= nv[2][j] &&
                                  v >= nv[2][j + 1] && v >= nv[2][j + 2];
                bits |= cand ? 1u << j : 0u;
            }
        }
        const int cnt = __popc(bits);
        int incl = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane == 63) wave_tot[wave] = incl;
        __syncthreads();
        int off = base_s + incl - cnt;
        for (int q = 0; q < wave; ++q) off += wave_tot[q];
        if (bits) {
            const float2 pv = P[((size_t)img * H + y) * W + x];
            const float inten = sqrtf(pv.x * pv.x + pv.y * pv.y);
#pragma unroll
            for (int j = 0; j < kR; ++j) {
                if (!(bits & (1u << j))) continue;
                if (off < row_cap) {
                    ulm_loc_t rec;
                    rec.plane = img / F;
                    rec.frame = img % F;
                    rec.iz = y;
                    rec.iu = x;
                    rec.z = ((float)(y * kR + i) + 0.5f) / kR - 0.5f;
                    rec.u = ((float)(x * kR + j) + 0.5f) / kR - 0.5f;
                    rec.ncc = vals[j];
                    rec.intensity = inten;
                    out[off] = rec;
                }
                ++off;
            }
        }
        __syncthreads();       // hs and wave_tot are rewritten by the next chunk
        if (t == 0) base_s += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
        __syncthreads();
    }
    if (t == 0) {
        row_cnt[(size_t)img * H + y] = min(base_s, row_cap);
        if (base_s > row_cap) atomicOr(status, kStatusCnnRow);
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
    for (int n0 = 0; n0 < n_img; n0 += batch) {
        const int nb = std::min(batch, n_img - n0);
        hipError_t e = cnn_images(P, fmax, x0, H * W, n0, nb, st);
        if (e != hipSuccess) return e;
        int last = 0;
        if ((e = run_forward<T>(params, x0, act, 2, (T *)(cws + L.wm), (T *)(cws + L.wt), nb, H, W,
                                st, &last)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(cnn_head_decode_kernel<T>, dim3(H, nb), dim3(256), 0, st, act[last],
                           params, P, thr, H, W, n0, F, staged, cnt, L.row_cap, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return launch_compact(cnt, off, n_img * H, count, staged, L.row_cap, locs, capacity, st);
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
