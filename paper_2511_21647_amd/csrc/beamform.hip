// Two-stage row-column beamforming to projection planes (paper Section II-A1,
// and the sub-block sum projection of Section II-A4).
//
// Stage 1 (das_stage1_kernel): per transmit, delay-and-sum of all receive
// elements into the reference slice S_k(u, z).  One work-group owns an 8 x 32
// pixel tile, one transmit and 16 frames: the delay, interpolation weight and
// phasor of each (pixel, element) pair are evaluated once and applied to all 16
// frames.  For each element the samples that the tile can reach are staged in
// LDS (double-buffered, next element's global loads in flight during the
// current element's arithmetic), so the gathers hit LDS, not the cache.
//
// Stage 2 (stage2_fir_kernel): extrapolation along the transmit direction,
// coherent compounding and slab projection collapse into one complex axial FIR
// per (transmit, slab): P(u, z) = sum_k sum_d H_k[d] S_k(u, z + d).
#include "common.h"

namespace ulm {

// Work-group remap so that consecutive logical work-groups land on the same
// XCD (the dispatcher deals work-groups round-robin over the 8 XCDs): the
// tiles that read the same channel data then share one L2.
__device__ inline int xcd_remap(int lin, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = lin & 7, s = lin >> 3;
    return x * q + min(x, r) + s;
}

template <int FB>
__global__ __launch_bounds__(kDasThreads) void das_stage1_kernel(
    const float2 *__restrict__ iq, float2 *__restrict__ S, const float *__restrict__ stx,
    const float2 *__restrict__ phz, Geometry g, int n_tu, int n_tz, int n_fb)
{
    const int n_wg = n_tu * n_tz * n_fb * 2 * g.n_angles;
    const int w = xcd_remap(blockIdx.x, n_wg);
    const int tile = w % (n_tu * n_tz);
    const int fb = (w / (n_tu * n_tz)) % n_fb;
    const int ok = w / (n_tu * n_tz * n_fb);
    const int o = ok / g.n_angles, k = ok % g.n_angles;
    const int tz = tile / n_tu, tu = tile % n_tu;

    const int t = threadIdx.x;
    const int iz = tz * kDasTileZ + t / kDasTileU;
    const int iu = tu * kDasTileU + t % kDasTileU;
    const bool valid = iz < g.nz && iu < g.nu;
    const int izc = min(iz, g.nz - 1), iuc = min(iu, g.nu - 1);
    const float z = g.z0 + izc * g.dz;
    const float u = g.u0 + iuc * g.du;
    const float stx_p = stx[k * g.nz + izc];

    // Tile extent (clamped to the grid) for the per-element sample window.
    const int iz_lo = tz * kDasTileZ, iu_lo = tu * kDasTileU;
    const int iu_hi = min(iu_lo + kDasTileU, g.nu) - 1;
    const float z_lo = g.z0 + iz_lo * g.dz;
    const float u_lo = g.u0 + iu_lo * g.du, u_hi = g.u0 + iu_hi * g.du;
    const float stx_lo = stx[k * g.nz + iz_lo];

    __shared__ float2 buf[2][FB][kDasLen];

    const size_t frame_stride = (size_t)2 * g.n_angles * g.n_elem * g.n_samp;
    const int f0 = fb * FB;
    const float2 *blk = iq + ((size_t)f0 * 2 * g.n_angles + (size_t)o * g.n_angles + k) *
                                 g.n_elem * g.n_samp;
    const float half_ap = 0.5f * (g.n_elem - 1);

    // First sample staged for element j: the smallest delay over the tile is at
    // its shallowest row and the column nearest to the element.
    auto window = [&](int j) -> int {
        const float ej = (j - half_ap) * g.pitch;
        const float dxn = fminf(fmaxf(ej, u_lo), u_hi) - ej;
        const float r = sqrtf(fmaf(z_lo, z_lo, dxn * dxn));
        return (int)floorf(fmaf(r, g.fs_over_c, stx_lo)) - 1;
    };

    constexpr int kPer = FB * kDasLen / kDasThreads;
    float2 pre[kPer];
    auto load = [&](int j, int s_lo) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = t + q * kDasThreads;
            const int f = e / kDasLen, s = e % kDasLen;
            const int gs = s_lo + s;
            float2 v = make_float2(0.f, 0.f);
            if (f0 + f < g.n_frames && gs >= 0 && gs < g.n_samp)
                v = blk[(size_t)f * frame_stride + (size_t)j * g.n_samp + gs];
            pre[q] = v;
        }
    };
    auto store = [&](int b) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = t + q * kDasThreads;
            buf[b][e / kDasLen][e % kDasLen] = pre[q];
        }
    };

    float2 acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = make_float2(0.f, 0.f);

    int s_lo = window(0);
    load(0, s_lo);
    store(0);
    __syncthreads();

    for (int j = 0; j < g.n_elem; ++j) {
        const int cur = j & 1;
        int s_next = 0;
        if (j + 1 < g.n_elem) {
            s_next = window(j + 1);
            load(j + 1, s_next);
        }
        // receive delay, fractional sample and phasor exp(i 2 pi f0 (r - z) / c)
        const float ej = (j - half_ap) * g.pitch;
        const float dx = u - ej;
        const float dx2 = dx * dx;
        const float r = sqrtf(fmaf(z, z, dx2));
        const float s = fmaf(r, g.fs_over_c, stx_p);
        const float fl = floorf(s);
        const float fr = s - fl;
        int idx = (int)fl - s_lo;
        idx = min(max(idx, 0), kDasLen - 2);
        float cyc = (dx2 / (r + z)) * g.f0_over_c;
        cyc -= rintf(cyc);
        float sn, cs;
        sincospif(2.0f * cyc, &sn, &cs);
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const float2 a = buf[cur][f][idx];
            const float2 b = buf[cur][f][idx + 1];
            const float xr = fmaf(fr, b.x - a.x, a.x);
            const float xi = fmaf(fr, b.y - a.y, a.y);
            acc[f].x = fmaf(cs, xr, fmaf(-sn, xi, acc[f].x));
            acc[f].y = fmaf(cs, xi, fmaf(sn, xr, acc[f].y));
        }
        if (j + 1 < g.n_elem) store(cur ^ 1);
        __syncthreads();
        s_lo = s_next;
    }

    if (!valid) return;
    const float2 ph = phz[k * g.nz + izc];
    const size_t plane = (size_t)g.nz * g.nu;
    float2 *dst = S + ((size_t)(o * g.n_angles + k) * g.n_frames) * plane + (size_t)iz * g.nu + iu;
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        if (f0 + f < g.n_frames) {
            float2 v;
            v.x = acc[f].x * ph.x - acc[f].y * ph.y;
            v.y = acc[f].x * ph.y + acc[f].y * ph.x;
            dst[(size_t)(f0 + f) * plane] = v;
        }
    }
}

__global__ __launch_bounds__(256) void stage2_fir_kernel(
    const float2 *__restrict__ S, float2 *__restrict__ P, const float2 *__restrict__ taps,
    Geometry g, int tap_min, int n_taps)
{
    const int c = threadIdx.x % kFirTileU;
    const int rg = threadIdx.x / kFirTileU;          // 4 groups of 8 rows
    const int u = blockIdx.x * kFirTileU + c;
    const int l0 = blockIdx.y * kFirTileZ;
    const int zf = blockIdx.z;                       // (o * B + b) * F + f
    const int f = zf % g.n_frames;
    const int ob = zf / g.n_frames;
    const int o = ob / g.n_blocks, b = ob % g.n_blocks;
    const size_t plane = (size_t)g.nz * g.nu;

    __shared__ float2 tile[kFirTileZ + kFirMaxTaps][kFirTileU];
    float2 acc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = make_float2(0.f, 0.f);

    const int rows = kFirTileZ + n_taps - 1;
    for (int k = 0; k < g.n_angles; ++k) {
        const float2 *src = S + ((size_t)(o * g.n_angles + k) * g.n_frames + f) * plane;
        for (int e = threadIdx.x; e < rows * kFirTileU; e += blockDim.x) {
            const int rr = e / kFirTileU, cc = e % kFirTileU;
            const int zz = l0 + tap_min + rr, uu = blockIdx.x * kFirTileU + cc;
            float2 v = make_float2(0.f, 0.f);
            if (zz >= 0 && zz < g.nz && uu < g.nu) v = src[(size_t)zz * g.nu + uu];
            tile[rr][cc] = v;
        }
        __syncthreads();
        const float2 *h = taps + (size_t)(k * g.n_blocks + b) * n_taps;
        for (int tt = 0; tt < n_taps; ++tt) {
            const float2 hv = h[tt];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const float2 x = tile[rg * 8 + r + tt][c];
                acc[r].x = fmaf(hv.x, x.x, fmaf(-hv.y, x.y, acc[r].x));
                acc[r].y = fmaf(hv.x, x.y, fmaf(hv.y, x.x, acc[r].y));
            }
        }
        __syncthreads();
    }
    if (u >= g.nu) return;
    float2 *dst = P + ((size_t)ob * g.n_frames + f) * plane;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int l = l0 + rg * 8 + r;
        if (l < g.nz) dst[(size_t)l * g.nu + u] = acc[r];
    }
}

hipError_t launch_stage1(const ulm_ctx *ctx, const float2 *iq, float2 *slices, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const int n_tu = cdiv(g.nu, kDasTileU), n_tz = cdiv(g.nz, kDasTileZ);
    const int n_fb = cdiv(g.n_frames, kDasFrames);
    const int n_wg = n_tu * n_tz * n_fb * 2 * g.n_angles;
    hipLaunchKernelGGL(das_stage1_kernel<kDasFrames>, dim3(n_wg), dim3(kDasThreads), 0, st, iq,
                       slices, ctx->tab.stx, ctx->tab.phz, g, n_tu, n_tz, n_fb);
    return hipGetLastError();
}

hipError_t launch_stage2(const ulm_ctx *ctx, const float2 *slices, float2 *proj, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    dim3 grid(cdiv(g.nu, kFirTileU), cdiv(g.nz, kFirTileZ), 2 * g.n_blocks * g.n_frames);
    hipLaunchKernelGGL(stage2_fir_kernel, grid, dim3(256), 0, st, slices, proj, ctx->tab.taps, g,
                       ctx->tab.tap_min, ctx->tab.n_taps);
    return hipGetLastError();
}

}  // namespace ulm
