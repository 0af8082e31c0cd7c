// XDoppler of the projection planes (paper Section II-A4: the filtered RC and
// CR stacks are cross-correlated over a window of three frames before
// localisation).  Both orientations' compounded volumes live on one voxel grid,
// so each slab plane gets, besides its own orientation's projection, the other
// orientation's volume sum-projected over the same slab onto the same plane
// (the cross projection).  For plane o, slab b, lateral column i (the other
// orientation's v = v_i):
//   Q_{o,b}(v_i, z) = sum_k sum_{u in b} S^{o'}_k(u, z + (v_i - v_ref) t_k)
//                     exp(i 4 pi f0 (v_i - v_ref) t_k / c)
// The shift and phase depend on v_i only, so the sum over the slab's u
// samples is taken first, once per (transmit, slab, frame, depth):
//   cross_profile_kernel  s_{k,b}(z) = sum_{u in b} S_k(u, z)
//   cross_project_kernel  Q(v_i, z) = sum_k w0_{k,i} s_{k,b}(z + n_{k,i})
//                                          + w1_{k,i} s_{k,b}(z + n_{k,i} + 1)
// with the linear-interpolation weights times the phase precomputed per
// (transmit, column) in FP64 on the host.  After both stacks are filtered,
//   xdoppler_kernel       out_f = sqrt(|sum_{t = f-h}^{f+h} P_t conj(Q_t)|)
// (frames outside the ensemble left out), written as a complex stack with zero
// imaginary part for the localisers.
#include "common.h"

#include <algorithm>

namespace ulm {

constexpr int kXdRowMax = 1024;     // plane width limit of the short-slab profile path

__device__ inline float2 wave_sum2(float2 v) {
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o);
        v.y += __shfl_xor(v.y, o);
    }
    return v;
}

// One wave per kXdRows consecutive slice rows (orientation, transmit, frame,
// depth): the sums of each row over each slab's u samples.  Slabs of 64 or more
// columns are summed by the whole wave (the next row's loads in flight while
// this row is reduced); narrower slabs by one lane each from an LDS copy of
// the row.
constexpr int kXdRows = 8;

__global__ __launch_bounds__(256) void cross_profile_kernel(const float2 *__restrict__ S,
                                                            float2 *__restrict__ prof, int rows,
                                                            int nu, int nz, int F, int B, int per)
{
    __shared__ float2 buf[4][kXdRowMax];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + w) * kXdRows;
    auto dst = [&](int row, int b) {
        const int z = row % nz, f = (row / nz) % F, ok = row / (nz * F);
        return prof + (((size_t)ok * B + b) * F + f) * nz + z;
    };
    if (per >= 64) {
        // the wave's rows are read together (their loads in flight at once),
        // then reduced
        for (int b = 0; b < B; ++b) {
            const int u0 = b * per, u1 = min((b + 1) * per, nu);
            float2 s[kXdRows];
#pragma unroll
            for (int r = 0; r < kXdRows; ++r) s[r] = make_float2(0.f, 0.f);
            for (int u = u0 + lane; u < u1; u += 64) {
#pragma unroll
                for (int r = 0; r < kXdRows; ++r) {
                    const int row = min(row0 + r, rows - 1);
                    const float2 v = S[(size_t)row * nu + u];
                    s[r].x += v.x;
                    s[r].y += v.y;
                }
            }
#pragma unroll
            for (int r = 0; r < kXdRows; ++r) {
                const float2 t = wave_sum2(s[r]);
                if (lane == 0 && row0 + r < rows) *dst(row0 + r, b) = t;
            }
        }
    } else {
        for (int r = 0; r < kXdRows; ++r) {
            const int row = row0 + r;
            const bool live = row < rows;
            const float2 *src = S + (size_t)(live ? row : 0) * nu;
            if (live)
                for (int u = lane; u < nu; u += 64) buf[w][u] = src[u];
            __syncthreads();
            if (live)
                for (int b = lane; b < B; b += 64) {
                    float2 s = make_float2(0.f, 0.f);
                    for (int u = b * per; u < min((b + 1) * per, nu); ++u) {
                        s.x += buf[w][u].x;
                        s.y += buf[w][u].y;
                    }
                    *dst(row, b) = s;
                }
            __syncthreads();
        }
    }
}

// One work-group per (plane o, slab b, frame f, band of kXdBand depths), one
// thread per column i: the K profiles of the other orientation's slab sums
// for frame f sit in LDS, the column's K (shift, weights) pairs in registers.
constexpr int kXdBand = 16;
constexpr int kXdMaxK = 32;

__global__ __launch_bounds__(1024) void cross_project_kernel(const float2 *__restrict__ prof,
                                                             float2 *__restrict__ Q,
                                                             const int *__restrict__ xn,
                                                             const float4 *__restrict__ xw, int K,
                                                             int B, int F, int nz, int nu,
                                                             int nmin, int nmax)
{
    extern __shared__ float2 pr[];                // [K][rows lo .. hi)
    const int bands = cdiv(nz, kXdBand);
    int wg = blockIdx.x;
    const int band = wg % bands;
    wg /= bands;
    const int f = wg % F;
    wg /= F;
    const int b = wg % B, o = wg / B;
    const int src_o = 1 - o;
    // the band's rows z0 .. z1 - 1 read profile rows z + n and z + n + 1, n in
    // [nmin, nmax] over every (transmit, column); rows outside [0, nz) are zero
    const int z0 = band * kXdBand, z1 = min(z0 + kXdBand, nz);
    const int lo = max(z0 + nmin, 0), hi = min(z1 + nmax + 1, nz);
    const int span = max(hi - lo, 0);
    for (int e = threadIdx.x; e < K * span; e += blockDim.x) {
        const int k = e / span, z = lo + e % span;
        pr[e] = prof[((((size_t)src_o * K + k) * B + b) * F + f) * nz + z];
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i >= nu) return;
    float2 *dst = Q + (((size_t)(o * B + b) * F + f) * nz) * nu + i;
    float2 acc[kXdBand];
#pragma unroll
    for (int r = 0; r < kXdBand; ++r) acc[r] = make_float2(0.f, 0.f);
    for (int k = 0; k < K; ++k) {
        const int n = xn[k * nu + i];
        const float4 wv = xw[k * nu + i];
        const float2 *row = pr + k * span - lo;
#pragma unroll
        for (int r = 0; r < kXdBand; ++r) {
            const int m = z0 + r + n;
            const float2 a = (m >= lo && m < hi) ? row[m] : make_float2(0.f, 0.f);
            const float2 c = (m + 1 >= lo && m + 1 < hi) ? row[m + 1] : make_float2(0.f, 0.f);
            acc[r].x += wv.x * a.x - wv.y * a.y + wv.z * c.x - wv.w * c.y;
            acc[r].y += wv.x * a.y + wv.y * a.x + wv.z * c.y + wv.w * c.x;
        }
    }
#pragma unroll
    for (int r = 0; r < kXdBand; ++r)
        if (z0 + r < z1) dst[(size_t)(z0 + r) * nu] = acc[r];
}

// One thread per pixel of a plane, walking the frames with the last W products
// P_t conj(Q_t) in registers.  `out` may be `P` itself: frame t is read before
// any output at or after frame t - h is written.
template <int W>
__global__ __launch_bounds__(256) void xdoppler_kernel(const float2 *P, const float2 *__restrict__ Q,
                                                       float2 *out, int F, int npix, int planes)
{
    constexpr int h = (W - 1) / 2;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)planes * npix) return;
    const int p = (int)(idx % npix);
    const size_t base = (idx / npix) * (size_t)F * npix + p;
    float2 ring[W];
#pragma unroll
    for (int j = 0; j < W; ++j) ring[j] = make_float2(0.f, 0.f);
    for (int t = 0; t < F + h; ++t) {
#pragma unroll
        for (int j = 0; j + 1 < W; ++j) ring[j] = ring[j + 1];
        float2 pr = make_float2(0.f, 0.f);
        if (t < F) {
            const float2 a = P[base + (size_t)t * npix], b = Q[base + (size_t)t * npix];
            pr = make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);   // a conj(b)
        }
        ring[W - 1] = pr;
        if (t >= h) {
            float2 s = make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                s.x += ring[j].x;
                s.y += ring[j].y;
            }
            out[base + (size_t)(t - h) * npix] = make_float2(sqrtf(hypotf(s.x, s.y)), 0.f);
        }
    }
}

bool cross_supported(const Geometry &g, int per) {
    return (per >= 64 || g.nu <= kXdRowMax) && g.nu <= 1024 && g.n_angles <= kXdMaxK &&
           (size_t)g.n_angles * g.nz * sizeof(float2) <= 64 * 1024;
}

hipError_t launch_cross(const ulm_ctx *ctx, const float2 *slices, float2 *prof, float2 *Q,
                        hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const int K = g.n_angles, B = g.n_blocks, F = g.n_frames;
    const int per = cdiv(g.nu, B);
    const int rows = 2 * K * F * g.nz;
    hipLaunchKernelGGL(cross_profile_kernel, dim3(cdiv(rows, 4 * kXdRows)), dim3(256), 0, st, slices,
                       prof, rows, g.nu, g.nz, F, B, per);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n_wg = (size_t)2 * B * F * cdiv(g.nz, kXdBand);
    const int threads = 64 * cdiv(g.nu, 64);
    hipLaunchKernelGGL(cross_project_kernel, dim3((unsigned)n_wg), dim3(threads),
                       sizeof(float2) * K * std::min(g.nz, kXdBand + ctx->tab.xd_nmax - ctx->tab.xd_nmin + 1),
                       st, prof, Q, ctx->tab.xd_n, ctx->tab.xd_w, K, B, F, g.nz, g.nu,
                       ctx->tab.xd_nmin, ctx->tab.xd_nmax);
    return hipGetLastError();
}

hipError_t launch_xdoppler(const ulm_ctx *ctx, const float2 *P, const float2 *Q, int window,
                           float2 *out, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const int npix = g.nz * g.nu, planes = g.n_planes;
    const size_t n = (size_t)planes * npix;
    const dim3 grid((unsigned)cdiv<size_t>(n, 256));
    switch (window) {
        case 1: hipLaunchKernelGGL(xdoppler_kernel<1>, grid, dim3(256), 0, st, P, Q, out, g.n_frames, npix, planes); break;
        case 3: hipLaunchKernelGGL(xdoppler_kernel<3>, grid, dim3(256), 0, st, P, Q, out, g.n_frames, npix, planes); break;
        case 5: hipLaunchKernelGGL(xdoppler_kernel<5>, grid, dim3(256), 0, st, P, Q, out, g.n_frames, npix, planes); break;
        case 7: hipLaunchKernelGGL(xdoppler_kernel<7>, grid, dim3(256), 0, st, P, Q, out, g.n_frames, npix, planes); break;
        default: hipLaunchKernelGGL(xdoppler_kernel<9>, grid, dim3(256), 0, st, P, Q, out, g.n_frames, npix, planes); break;
    }
    return hipGetLastError();
}

}  // namespace ulm
