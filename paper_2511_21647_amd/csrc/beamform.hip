// Stage 2 of the two-stage row-column beamforming (paper Section II-A1, and
// the sub-block sum projection of Section II-A4): extrapolation along the
// transmit direction, coherent compounding and slab projection collapse into
// one complex axial FIR per (transmit, slab):
//   P(u, z) = sum_k sum_d H_k[d] S_k(u, z + d).
#include "common.h"

#include <stdint.h>

namespace ulm {

// G slabs per work-group: for each transmit the slice tile covers the union of
// the G slabs' tap ranges and is read from HBM once for all of them.
template <int G>
__global__ __launch_bounds__(256, 4) void stage2_fir_kernel(
    const float2 *__restrict__ S, float2 *__restrict__ P, const float2 *__restrict__ taps,
    const int2 *__restrict__ meta, Geometry g, int max_taps)
{
    // logical work-group order ((o F + f) tiles + tile) NG + slab group: the slab
    // groups of one tile and frame run back to back on one XCD and share its L2
    // copy of the slice tiles
    const int NG = cdiv(g.n_blocks, G);
    const int n_tu = cdiv(g.nu, kFirTileU), tiles = n_tu * cdiv(g.nz, kFirTileZ);
    const int n_wg = 2 * g.n_frames * tiles * NG;
    int lw = xcd_remap(blockIdx.x, n_wg);
    const int b0 = (lw % NG) * G;
    lw /= NG;
    const int ti = lw % tiles;
    lw /= tiles;
    const int f = lw % g.n_frames, o = lw / g.n_frames;
    const int tu = ti % n_tu, tz = ti / n_tu;
    const int c = threadIdx.x % kFirTileU;
    const int rg = threadIdx.x / kFirTileU;          // 8 groups of 8 rows
    const int u = tu * kFirTileU + c;
    const int l0 = tz * kFirTileZ;
    const size_t plane = (size_t)g.nz * g.nu;

    __shared__ float2 tile[kFirTileZ + kFirMaxTaps][kFirTileU];
    float2 acc[G][8];
#pragma unroll
    for (int gb = 0; gb < G; ++gb)
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[gb][r] = make_float2(0.f, 0.f);

    // union of the group's tap offsets for transmit k: [lo, hi)
    auto span_of = [&](int k, int &lo, int &hi) {
        lo = INT32_MAX;
        hi = INT32_MIN;
#pragma unroll
        for (int gb = 0; gb < G; ++gb)
            if (b0 + gb < g.n_blocks) {
                const int2 m = meta[k * g.n_blocks + b0 + gb];
                lo = min(lo, m.x);
                hi = max(hi, m.x + m.y);
            }
    };
    // the slice tile of transmit k (rows l0 + lo .. , one row past the last tap
    // of each window): element e = t + 256 i of the tile goes through pre[i]
    constexpr int kPer = ((kFirTileZ + kFirMaxTaps) * kFirTileU + 255) / 256;
    float2 pre[kPer];
    auto fetch = [&](int k, int lo, int rows) {
        const float2 *src = S + ((size_t)(o * g.n_angles + k) * g.n_frames + f) * plane;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int rr = e / kFirTileU, cc = e % kFirTileU;
            const int zz = l0 + lo + rr, uu = tu * kFirTileU + cc;
            pre[i] = make_float2(0.f, 0.f);
            if (rr < rows && zz >= 0 && zz < g.nz && uu < g.nu) pre[i] = src[(size_t)zz * g.nu + uu];
        }
    };
    auto stash = [&](int rows) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < rows * kFirTileU) tile[e / kFirTileU][e % kFirTileU] = pre[i];
        }
    };
    auto filter = [&](int k, int lo_k) {
#pragma unroll
        for (int gb = 0; gb < G; ++gb) {
            if (b0 + gb >= g.n_blocks) continue;
            const int2 m = meta[k * g.n_blocks + b0 + gb];
            // 8 consecutive output rows per thread: a rotating window of 8 input rows
            // in registers, so each tap costs one LDS read instead of eight
            const float2 *h = taps + (size_t)(k * g.n_blocks + b0 + gb) * max_taps;
            const int base = rg * 8 + (m.x - lo_k);
            float2 win[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) win[r] = tile[base + r][c];
            auto step = [&](int tt, int uu) {   // tap tt = 8 q + uu
                const float2 hv = h[tt];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const float2 x = win[(r + uu) & 7];
                    acc[gb][r].x = fmaf(hv.x, x.x, fmaf(-hv.y, x.y, acc[gb][r].x));
                    acc[gb][r].y = fmaf(hv.x, x.y, fmaf(hv.y, x.x, acc[gb][r].y));
                }
                win[uu] = tile[base + 8 + tt][c];     // row base + tt is no longer needed
            };
            int tt = 0;
            for (; tt + 8 <= m.y; tt += 8) {
#pragma unroll
                for (int uu = 0; uu < 8; ++uu) step(tt + uu, uu);
            }
#pragma unroll
            for (int uu = 0; uu < 8; ++uu)
                if (tt + uu < m.y) step(tt + uu, uu);
        }
    };
    int lo, hi;
    if constexpr (G == 1) {
        // one slab: the next transmit's tile is loaded while this one is filtered
        span_of(0, lo, hi);
        fetch(0, lo, kFirTileZ + (hi - lo));
        for (int k = 0; k < g.n_angles; ++k) {
            stash(kFirTileZ + (hi - lo));
            __syncthreads();
            const int lo_k = lo;
            if (k + 1 < g.n_angles) {
                span_of(k + 1, lo, hi);
                fetch(k + 1, lo, kFirTileZ + (hi - lo));
            }
            filter(k, lo_k);
            __syncthreads();
        }
    } else {
        // G slabs hold G x 8 accumulators: no registers to spare for a prefetch
        for (int k = 0; k < g.n_angles; ++k) {
            span_of(k, lo, hi);
            const int rows = kFirTileZ + (hi - lo);
            const float2 *src = S + ((size_t)(o * g.n_angles + k) * g.n_frames + f) * plane;
            for (int e = threadIdx.x; e < rows * kFirTileU; e += blockDim.x) {
                const int rr = e / kFirTileU, cc = e % kFirTileU;
                const int zz = l0 + lo + rr, uu = tu * kFirTileU + cc;
                float2 v = make_float2(0.f, 0.f);
                if (zz >= 0 && zz < g.nz && uu < g.nu) v = src[(size_t)zz * g.nu + uu];
                tile[rr][cc] = v;
            }
            __syncthreads();
            filter(k, lo);
            __syncthreads();
        }
    }
    if (u >= g.nu) return;
#pragma unroll
    for (int gb = 0; gb < G; ++gb) {
        if (b0 + gb >= g.n_blocks) continue;
        float2 *dst = P + ((size_t)(o * g.n_blocks + b0 + gb) * g.n_frames + f) * plane;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int l = l0 + rg * 8 + r;
            if (l < g.nz) dst[(size_t)l * g.nu + u] = acc[gb][r];
        }
    }
}

hipError_t launch_stage2(const ulm_ctx *ctx, const float2 *slices, float2 *proj, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const int G = ctx->tab.fir_group;
    const size_t n_wg = (size_t)2 * g.n_frames * cdiv(g.nu, kFirTileU) * cdiv(g.nz, kFirTileZ) *
                        cdiv(g.n_blocks, G);
    if (n_wg > (size_t)INT32_MAX) return hipErrorInvalidConfiguration;
    if (G == kFirGroup)
        hipLaunchKernelGGL(stage2_fir_kernel<kFirGroup>, dim3((unsigned)n_wg), dim3(256), 0, st,
                           slices, proj, ctx->tab.taps, ctx->tab.tap_meta, g, ctx->tab.n_taps);
    else
        hipLaunchKernelGGL(stage2_fir_kernel<1>, dim3((unsigned)n_wg), dim3(256), 0, st, slices,
                           proj, ctx->tab.taps, ctx->tab.tap_meta, g, ctx->tab.n_taps);
    return hipGetLastError();
}

}  // namespace ulm
