// NCC microbubble localisation (paper Section II-A4) on filtered planes.
//
//   frame_max_kernel   per-(plane, frame) maximum of the envelope |P|, the
//                      reference of the intensity threshold
//   ncc_detect_kernel  one work-group per band of 16 rows x full width: envelope
//                      tile with halo in LDS, two separable passes (Fig. 1g) of
//                      three sums (template, box, box of squares), zero-mean NCC,
//                      3x3 regional maxima with raster tie-break, thresholds,
//                      3-point Gaussian sub-pixel fit, and an in-band compaction
//                      in raster order (wave ballots + a block scan)
//   loc_scan_kernel    exclusive scan of the per-band counts
//   loc_scatter_kernel copies each band's records to its output offset
// Output order is (plane, frame, row, column) without any sort: bands are full
// width and are laid out in that order.
#include "common.h"

#include <math.h>

namespace ulm {

struct NccParams {
    int half;             // template half width h
    float kbar;           // mean of the template
    float inv_w;          // 1 / size^2
    float inv_sk;         // 1 / sqrt(sum (K - Kbar)^2)
    float tau, alpha;
    float gz[2 * kNccMaxHalf + 1], gu[2 * kNccMaxHalf + 1];
};

__global__ __launch_bounds__(256) void frame_max_kernel(const float2 *__restrict__ P,
                                                        float *__restrict__ fmax_out, int npix)
{
    const float2 *src = P + (size_t)blockIdx.x * npix;
    float m = 0.f;
    // eight loads in flight per thread (the launch is one work-group per image)
    int i = threadIdx.x;
    for (; i + 7 * 256 < npix; i += 8 * 256) {
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[i + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) m = fmaxf(m, sqrtf(v[u].x * v[u].x + v[u].y * v[u].y));
    }
    for (; i < npix; i += 256) {
        const float2 v = src[i];
        m = fmaxf(m, sqrtf(v.x * v.x + v.y * v.y));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) fmax_out[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__device__ inline float subpix(float nm, float n0, float np) {
    float d;
    if (nm > 0.f && n0 > 0.f && np > 0.f) {
        const float lm = logf(nm), l0 = logf(n0), lp = logf(np);
        const float den = 2.f * (lm - 2.f * l0 + lp);
        d = den < 0.f ? (lm - lp) / den : 0.f;
    } else {
        const float den = 2.f * (nm - 2.f * n0 + np);
        d = den < 0.f ? (nm - np) / den : 0.f;
    }
    return fminf(fmaxf(d, -0.5f), 0.5f);
}

// Peak test, sub-pixel fit and raster-order compaction of one band, from the
// band's NCC rows (with a halo row above and below) in LDS.  Thread t tests the
// raster run [t R, t R + R) of the band's pixels and counts its peaks; one
// block-wide prefix sum of the counts gives every thread its output offset, so
// the records come out in raster order with a single barrier.
__device__ void detect_band(const float *ncc, const float2 *__restrict__ src,
                            const float *__restrict__ fmax_in, ulm_loc_t *__restrict__ staged,
                            int *__restrict__ band_cnt, const NccParams &prm, int nz, int nu,
                            int F, int bands, int band_cap, int band, int f, int plane)
{
    const int W_out = nu + 2;
    const int r0 = band * kNccBand;
    __shared__ int wave_tot[16];
    const float thr_i = prm.alpha * fmax_in[plane * F + f];
    const int rows = min(kNccBand, nz - r0);
    const int npx = rows * nu;
    ulm_loc_t *out = staged + ((size_t)(plane * F + f) * bands + band) * band_cap;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    const int R = (npx + blockDim.x - 1) / blockDim.x;
    const int e0 = min((int)threadIdx.x * R, npx), e1 = min(e0 + R, npx);

    // NCC threshold, 3x3 regional maximum (raster tie-break), then the intensity
    // threshold (its global read only for the few regional maxima); (rr, cc) is
    // the position in the ncc array
    auto is_peak_at = [&](int rr, int cc, float &I) {
        const float n0 = ncc[rr * W_out + cc];
        if (!(n0 >= prm.tau)) return false;
        const float *up = ncc + (rr - 1) * W_out + cc;
        const float *mid = ncc + rr * W_out + cc;
        const float *dn = ncc + (rr + 1) * W_out + cc;
        if (!(n0 > up[-1] && n0 > up[0] && n0 > up[1] && n0 > mid[-1] && n0 >= mid[1] &&
              n0 >= dn[-1] && n0 >= dn[0] && n0 >= dn[1]))
            return false;
        const float2 x = src[(size_t)(r0 + rr - 1) * nu + (cc - 1)];
        I = sqrtf(x.x * x.x + x.y * x.y);
        return I >= thr_i;
    };
    auto is_peak = [&](int e, float &I) { return is_peak_at(e / nu + 1, e % nu + 1, I); };
    unsigned long long mask = 0ull;                           // peaks among the run's first 64
    int cnt = 0;
    {
        // the run's position advanced along the raster (one division per thread)
        int rr = e0 / nu + 1, cc = e0 % nu + 1;
        for (int e = e0; e < e1; ++e) {
            float I;
            if (is_peak_at(rr, cc, I)) {
                if (e - e0 < 64) mask |= 1ull << (e - e0);
                ++cnt;
            }
            if (++cc > nu) {
                cc = 1;
                ++rr;
            }
        }
    }
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    int off = incl - cnt, total = 0;
    for (int q = 0; q < nw; ++q) {
        if (q < wv) off += wave_tot[q];
        total += wave_tot[q];
    }
    auto emit = [&](int e, float I) {
        const int rr = e / nu + 1, cc = e % nu + 1;
        const int z = r0 + rr - 1, u = cc - 1;
        const float *up = ncc + (rr - 1) * W_out + cc;
        const float *mid = ncc + rr * W_out + cc;
        const float *dn = ncc + (rr + 1) * W_out + cc;
        const float n0 = mid[0];
        const float dz = (z > 0 && z < nz - 1) ? subpix(up[0], n0, dn[0]) : 0.f;
        const float du = (u > 0 && u < nu - 1) ? subpix(mid[-1], n0, mid[1]) : 0.f;
        ulm_loc_t rec;
        rec.plane = plane;
        rec.frame = f;
        rec.iz = z;
        rec.iu = u;
        rec.z = (float)z + dz;
        rec.u = (float)u + du;
        rec.ncc = n0;
        rec.intensity = I;
        out[off++] = rec;
    };
    while (mask) {
        const int i = __ffsll((long long)mask) - 1;
        mask &= mask - 1ull;
        float I;
        is_peak(e0 + i, I);                                   // recomputes I for the record
        emit(e0 + i, I);
    }
    for (int e = e0 + 64; e < e1; ++e) {                      // runs longer than 64 pixels
        float I;
        if (is_peak(e, I)) emit(e, I);
    }
    if (threadIdx.x == 0) band_cnt[(plane * F + f) * bands + band] = total;
}

// Dynamic LDS: img [R_in][W_in] (reused for ncc [kNccBand+2][nu+2]), then
// Vg, V1, V2 [kNccBand+2][W_in].
__global__ __launch_bounds__(256) void ncc_detect_kernel(
    const float2 *__restrict__ P, const float *__restrict__ fmax_in, ulm_loc_t *__restrict__ staged,
    int *__restrict__ band_cnt, NccParams prm, int nz, int nu, int F, int bands, int band_cap)
{
    extern __shared__ float smem[];
    const int band = blockIdx.x, f = blockIdx.y, plane = blockIdx.z;
    const int h = prm.half;
    const int R_out = kNccBand + 2;                 // NCC rows with a halo of 1
    const int R_in = R_out + 2 * h;
    const int W_in = nu + 2 + 2 * h;
    const int W_out = nu + 2;
    float *img = smem;
    float *Vg = smem + (size_t)R_in * W_in;
    float *V1 = Vg + (size_t)R_out * W_in;
    float *V2 = V1 + (size_t)R_out * W_in;
    float *ncc = img;                               // after the vertical pass

    const int r0 = band * kNccBand;                 // first output row of the band
    const float2 *src = P + ((size_t)plane * F + f) * (size_t)nz * nu;

    for (int e = threadIdx.x; e < R_in * W_in; e += blockDim.x) {
        const int rr = e / W_in, cc = e % W_in;
        const int z = r0 - 1 - h + rr, u = cc - 1 - h;
        float v = 0.f;
        if (z >= 0 && z < nz && u >= 0 && u < nu) {
            const float2 x = src[(size_t)z * nu + u];
            v = sqrtf(x.x * x.x + x.y * x.y);
        }
        img[e] = v;
    }
    __syncthreads();
    const int S = 2 * h + 1;
    for (int e = threadIdx.x; e < R_out * W_in; e += blockDim.x) {
        const int rr = e / W_in, cc = e % W_in;
        float sg = 0.f, s1 = 0.f, s2 = 0.f;
        for (int a = 0; a < S; ++a) {
            const float x = img[(rr + a) * W_in + cc];
            sg = fmaf(prm.gz[a], x, sg);
            s1 += x;
            s2 = fmaf(x, x, s2);
        }
        Vg[e] = sg;
        V1[e] = s1;
        V2[e] = s2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R_out * W_out; e += blockDim.x) {
        const int rr = e / W_out, cc = e % W_out;
        const int z = r0 - 1 + rr, u = cc - 1;
        float out = -INFINITY;                      // outside the image: ignored by the peak test
        if (z >= 0 && z < nz && u >= 0 && u < nu) {
            float sik = 0.f, si = 0.f, si2 = 0.f;
            const int base = rr * W_in + cc;
            for (int b = 0; b < S; ++b) {
                sik = fmaf(prm.gu[b], Vg[base + b], sik);
                si += V1[base + b];
                si2 += V2[base + b];
            }
            const float num = sik - prm.kbar * si;
            const float var = si2 - si * si * prm.inv_w;
            out = var > 1e-6f * si2 ? num * prm.inv_sk * rsqrtf(var) : 0.f;
        }
        ncc[e] = out;
    }
    __syncthreads();

    detect_band(ncc, src, fmax_in, staged, band_cnt, prm, nz, nu, F, bands, band_cap, band, f,
                plane);
}

// Register-column form of the same computation, for images up to 512 - 2 - 2H
// columns wide, launched with one thread per input column (the block rounded
// up to whole waves): thread t keeps column t's 18 + 2H envelope values in
// registers; each output row's vertical sums go through a small
// double-buffered LDS row, and the NCC rows of the band stay in LDS for the
// peak test.  About 27 KB of LDS per work-group at the paper's width (against
// ~91 KB for the staged form), so five work-groups share a CU.
template <int H>
__global__ __launch_bounds__(512) void ncc_band_kernel(
    const float2 *__restrict__ P, const float *__restrict__ fmax_in, ulm_loc_t *__restrict__ staged,
    int *__restrict__ band_cnt, NccParams prm, int nz, int nu, int F, int bands, int band_cap)
{
    constexpr int S = 2 * H + 1;
    constexpr int R_out = kNccBand + 2;
    constexpr int R_in = R_out + 2 * H;
    extern __shared__ float smem[];
    const int band = blockIdx.x, f = blockIdx.y, plane = blockIdx.z;
    const int W_in = nu + 2 + 2 * H, W_out = nu + 2;
    float *V = smem;                                // [2][3][W_in]
    float *ncc = smem + 6 * W_in;                   // [R_out][W_out]
    const int t = threadIdx.x;
    const int r0 = band * kNccBand;
    const float2 *src = P + ((size_t)plane * F + f) * (size_t)nz * nu;

    float col[R_in];
    {
        const int u = t - 1 - H;
        const bool cu = t < W_in && u >= 0 && u < nu;
#pragma unroll
        for (int rr = 0; rr < R_in; ++rr) {
            const int z = r0 - 1 - H + rr;
            float v = 0.f;
            if (cu && z >= 0 && z < nz) {
                const float2 x = src[(size_t)z * nu + u];
                v = sqrtf(x.x * x.x + x.y * x.y);
            }
            col[rr] = v;
        }
    }
#pragma unroll
    for (int rr = 0; rr < R_out; ++rr) {
        float *Vb = V + (rr & 1) * 3 * W_in;
        if (t < W_in) {
            float sg = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int a = 0; a < S; ++a) {
                const float x = col[rr + a];
                sg = fmaf(prm.gz[a], x, sg);
                s1 += x;
                s2 = fmaf(x, x, s2);
            }
            Vb[t] = sg;
            Vb[W_in + t] = s1;
            Vb[2 * W_in + t] = s2;
        }
        __syncthreads();
        const int z = r0 - 1 + rr;
        for (int co = t; co < W_out; co += blockDim.x) {
            const int u = co - 1;
            float out = -INFINITY;                  // outside the image: ignored by the peak test
            if (z >= 0 && z < nz && u >= 0 && u < nu) {
                float sik = 0.f, si = 0.f, si2 = 0.f;
#pragma unroll
                for (int b = 0; b < S; ++b) {
                    sik = fmaf(prm.gu[b], Vb[co + b], sik);
                    si += Vb[W_in + co + b];
                    si2 += Vb[2 * W_in + co + b];
                }
                const float num = sik - prm.kbar * si;
                const float var = si2 - si * si * prm.inv_w;
                out = var > 1e-6f * si2 ? num * prm.inv_sk * rsqrtf(var) : 0.f;
            }
            ncc[rr * W_out + co] = out;
        }
    }
    __syncthreads();
    detect_band(ncc, src, fmax_in, staged, band_cnt, prm, nz, nu, F, bands, band_cap, band, f,
                plane);
}

// Exclusive scan of n counts by one work-group; writes the total to *count.
__global__ __launch_bounds__(1024) void loc_scan_kernel(const int *__restrict__ cnt,
                                                        int *__restrict__ off, int n,
                                                        int *__restrict__ count)
{
    // passes of 4096 counts, 4 consecutive ones per thread: each wave scans its
    // threads' sums with lane shuffles, the 16 wave totals meet in LDS (double-
    // buffered by pass parity: one barrier per pass), and a running carry links
    // the passes; the next pass's counts are loaded during this one
    __shared__ int wtot[2][16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    auto load4 = [&](int b0, int (&v)[4]) {
        const int i0 = b0 + 4 * t;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = i0 + q < n ? cnt[i0 + q] : 0;
    };
    int cur[4], nxt[4];
    load4(0, cur);
    int carry = 0, par = 0;
    for (int b0 = 0; b0 < n; b0 += 4096) {
        load4(b0 + 4096, nxt);
        const int sum = cur[0] + cur[1] + cur[2] + cur[3];
        int incl = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        if (lane == 63) wtot[par][wv] = incl;
        __syncthreads();
        int base = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int x = wtot[par][q];
            if (q < wv) base += x;
            tot += x;
        }
        int run = carry + base + incl - sum;
        const int i0 = b0 + 4 * t;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (i0 + q < n) off[i0 + q] = run;
            run += cur[q];
        }
        carry += tot;
        par ^= 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
    }
    if (t == 0) *count = carry;
}

__global__ __launch_bounds__(256) void loc_scatter_kernel(
    const ulm_loc_t *__restrict__ staged, const int *__restrict__ cnt, const int *__restrict__ off,
    ulm_loc_t *__restrict__ locs, int capacity, int band_cap)
{
    const int slot = blockIdx.x;
    const int n = cnt[slot], o = off[slot];
    const ulm_loc_t *src = staged + (size_t)slot * band_cap;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (o + i < capacity) locs[o + i] = src[i];
}

__global__ void density_kernel(const ulm_loc_t *__restrict__ locs, const int *__restrict__ count,
                               int capacity, int up, int nz, int nu, int planes,
                               uint32_t *__restrict__ dens)
{
    const int n = min(*count, capacity);
    const int W = nu * up, H = nz * up;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const ulm_loc_t r = locs[i];
        const int bz = (int)floorf((r.z + 0.5f) * up);
        const int bu = (int)floorf((r.u + 0.5f) * up);
        if (r.plane < 0 || r.plane >= planes || bz < 0 || bz >= H || bu < 0 || bu >= W) continue;
        atomicAdd(&dens[((size_t)r.plane * H + bz) * W + bu], 1u);
    }
}

size_t ncc_lds_bytes(int nu, int half) {
    const size_t R_out = kNccBand + 2, R_in = R_out + 2 * half, W_in = nu + 2 + 2 * half;
    const size_t img = std::max(R_in * W_in, R_out * (size_t)(nu + 2));
    return (img + 3 * R_out * W_in) * sizeof(float);
}

NccParams make_ncc_params(const ulm_ctx *ctx) {
    const ulm_config_t &c = ctx->cfg;
    NccParams p{};
    const int h = (c.ncc_size - 1) / 2;
    p.half = h;
    double sz = 0, su = 0;
    double gz[2 * kNccMaxHalf + 1], gu[2 * kNccMaxHalf + 1];
    for (int a = -h; a <= h; ++a) {
        gz[a + h] = exp(-(double)a * a / (2.0 * c.sigma_z * c.sigma_z));
        gu[a + h] = exp(-(double)a * a / (2.0 * c.sigma_u * c.sigma_u));
        sz += gz[a + h];
        su += gu[a + h];
        p.gz[a + h] = (float)gz[a + h];
        p.gu[a + h] = (float)gu[a + h];
    }
    const double W = (double)c.ncc_size * c.ncc_size;
    const double kbar = sz * su / W;
    double sk = 0;
    for (int a = 0; a < c.ncc_size; ++a)
        for (int b = 0; b < c.ncc_size; ++b) {
            const double d = gz[a] * gu[b] - kbar;
            sk += d * d;
        }
    p.kbar = (float)kbar;
    p.inv_w = (float)(1.0 / W);
    p.inv_sk = (float)(1.0 / sqrt(sk));
    p.tau = (float)c.tau_ncc;
    p.alpha = (float)c.alpha;
    return p;
}

hipError_t launch_localize(const ulm_ctx *ctx, const float2 *filt, ulm_loc_t *locs, int capacity,
                           int *count, char *ws, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const Workspace &w = ctx->ws;
    const int npix = g.nz * g.nu, F = g.n_frames, planes = g.n_planes;
    float *fmx = (float *)(ws + w.fmax);
    int *bcnt = (int *)(ws + w.band_cnt);
    int *boff = (int *)(ws + w.band_off);
    ulm_loc_t *staged = (ulm_loc_t *)(ws + w.staged);
    hipLaunchKernelGGL(frame_max_kernel, dim3(planes * F), dim3(256), 0, st, filt, fmx, npix);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const NccParams prm = make_ncc_params(ctx);
    const dim3 grid(w.bands, F, planes);
    const int W_in = g.nu + 2 + 2 * prm.half;
    if (W_in <= 512) {
        const size_t lds = (6 * (size_t)W_in + (size_t)(kNccBand + 2) * (g.nu + 2)) * sizeof(float);
        const int threads = 64 * cdiv(W_in, 64);            // one per input column, <= 512
#define ULM_NCC_BAND(HH)                                                                          \
    case HH:                                                                                      \
        hipLaunchKernelGGL(ncc_band_kernel<HH>, grid, dim3(threads), lds, st, filt, fmx, staged, bcnt, \
                           prm, g.nz, g.nu, F, w.bands, w.band_cap);                              \
        break;
        switch (prm.half) {
            ULM_NCC_BAND(1)
            ULM_NCC_BAND(2)
            ULM_NCC_BAND(3)
            ULM_NCC_BAND(4)
            ULM_NCC_BAND(5)
            ULM_NCC_BAND(6)
            ULM_NCC_BAND(7)
            default: return hipErrorInvalidValue;
        }
#undef ULM_NCC_BAND
    } else {
        const size_t lds = ncc_lds_bytes(g.nu, prm.half);
        hipLaunchKernelGGL(ncc_detect_kernel, grid, dim3(256), lds, st, filt, fmx, staged, bcnt,
                           prm, g.nz, g.nu, F, w.bands, w.band_cap);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nslots = planes * F * w.bands;
    hipLaunchKernelGGL(loc_scan_kernel, dim3(1), dim3(1024), 0, st, bcnt, boff, nslots, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(loc_scatter_kernel, dim3(nslots), dim3(256), 0, st, staged, bcnt, boff,
                       locs, capacity, w.band_cap);
    return hipGetLastError();
}

hipError_t launch_frame_max(const float2 *P, float *fmax, int n_img, int npix, hipStream_t st)
{
    hipLaunchKernelGGL(frame_max_kernel, dim3(n_img), dim3(256), 0, st, P, fmax, npix);
    return hipGetLastError();
}

// Exclusive scan of n counts into off, the total into *count.
hipError_t launch_scan(const int *cnt, int *off, int n, int *count, hipStream_t st)
{
    hipLaunchKernelGGL(loc_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, off, n, count);
    return hipGetLastError();
}

// Exclusive scan of per-slot counts, then each slot's records to its offset.
hipError_t launch_compact(const int *cnt, int *off, int nslots, int *count, const ulm_loc_t *staged,
                          int cap, ulm_loc_t *locs, int capacity, hipStream_t st)
{
    hipLaunchKernelGGL(loc_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, off, nslots, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loc_scatter_kernel, dim3(nslots), dim3(256), 0, st, staged, cnt, off, locs,
                       capacity, cap);
    return hipGetLastError();
}

hipError_t launch_density(const ulm_ctx *ctx, const ulm_loc_t *locs, const int *count,
                          int capacity, int up, uint32_t *dens, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    hipLaunchKernelGGL(density_kernel, dim3(1024), dim3(256), 0, st, locs, count, capacity, up,
                       g.nz, g.nu, g.n_planes, dens);
    return hipGetLastError();
}


}  // namespace ulm
