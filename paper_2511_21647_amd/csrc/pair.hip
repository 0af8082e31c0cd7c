// Pairing of the two orthogonal projections' 2D localisations into 3D MB
// positions (paper Section II-A4): an XZ localisation i and a YZ localisation
// j of the same frame are candidates when |z_i - z_j| <= 1 voxel and the
// intensity ratio I_i / I_j lies in [0.9, 1.11]; pairs are the mutual minima of
// the ratio's distance from 1, max(rho, 1/rho) (ties to the smaller record
// index); the 3D position takes x from XZ, y from YZ and the mean z.  With B
// slabs per orientation, XZ records of slab b pair only with YZ records whose
// y lies in slab b, and their x must lie in the YZ record's slab.
//
//   pair_bounds_kernel  record range of every (plane, frame) in the sorted list
//   pair_best_kernel    every record's best candidate (one work-group per
//                       (frame, plane))
//   pair_count_kernel   mutual pairs per (frame, XZ plane)
//   launch_scan         their offsets, XZ planes fastest (the localisers' scan)
//   pair_write_kernel   the pairs of each (frame, XZ plane); records are sorted by
//                       plane, so (frame, plane) order is (frame, XZ index) order
#include "common.h"

#include <math.h>

#include <algorithm>

namespace ulm {

struct PairArgs {
    const ulm_loc_t *locs;
    int n;                  // records in use: min(count, capacity)
    int F, B, per;          // frames, slabs per orientation, slab width in pixels
    const int *bounds;      // [2B][F][2]
    int *best;              // [n]
    int *cnt, *off;         // [F][B]
};

// slab of a plane coordinate (pixel units), or -1 outside [-0.5, 1e6)
__device__ inline int slab_of(float pix, int per) {
    if (!(pix >= -0.5f && pix < 1e6f)) return -1;
    return (int)floorf(pix + 0.5f) / per;
}

__device__ inline int key_of(const ulm_loc_t &r, int F) { return r.plane * F + r.frame; }

__global__ void pair_bounds_kernel(const ulm_loc_t *__restrict__ locs, const int *__restrict__ count,
                                   int capacity, int nkeys, int F, int *__restrict__ bounds)
{
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= nkeys) return;
    const int n = min(*count, capacity);
    auto lower = [&](int k) {          // first record with key >= k
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key_of(locs[mid], F) < k) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    bounds[2 * key] = lower(key);
    bounds[2 * key + 1] = lower(key + 1);
}

// cost of pairing an XZ record with a YZ record, each given as (z, u, ncc,
// intensity), or +inf if they are not candidates (the slab test is separate)
__device__ inline float pair_cost(float4 xz, float4 yz) {
    if (!(fabsf(xz.x - yz.x) <= 1.0f)) return INFINITY;
    if (!(xz.w > 0.f && yz.w > 0.f)) return INFINITY;
    const float rho = xz.w / yz.w;
    if (!(rho >= 0.9f && rho <= 1.11f)) return INFINITY;
    return fmaxf(rho, yz.w / xz.w);
}

// (z, u, ncc, intensity) of record r: the second 16 bytes of the record
__device__ inline float4 loc_zuni(const ulm_loc_t *locs, int r) {
    return *reinterpret_cast<const float4 *>(&locs[r].z);
}

__global__ __launch_bounds__(256) void pair_best_kernel(PairArgs a)
{
    const int f = blockIdx.x, p = blockIdx.y;
    const int lo = a.bounds[2 * (p * a.F + f)], hi = a.bounds[2 * (p * a.F + f) + 1];
    const bool xz = p < a.B;
    // with slabs, a candidate's u must lie in this plane's slab; the record's own
    // u picks the one segment of the other orientation that can hold its partner
    const int want = xz ? p : p - a.B;
    for (int r = lo + threadIdx.x; r < hi; r += blockDim.x) {
        const float4 me = loc_zuni(a.locs, r);
        int q;
        if (a.B == 1) {
            q = xz ? 1 : 0;
        } else {
            const int sl = slab_of(me.y, a.per);
            if (sl < 0 || sl >= a.B) {       // outside every slab: no partner
                a.best[r] = -1;
                continue;
            }
            q = xz ? a.B + sl : sl;
        }
        const int clo = a.bounds[2 * (q * a.F + f)], chi = a.bounds[2 * (q * a.F + f) + 1];
        float bc = INFINITY;
        int bi = -1;
#pragma unroll 4
        for (int c = clo; c < chi; ++c) {
            const float4 o = loc_zuni(a.locs, c);
            float cost = xz ? pair_cost(me, o) : pair_cost(o, me);
            if (a.B > 1 && slab_of(o.y, a.per) != want) cost = INFINITY;
            if (cost < bc) {            // strict: the first (smallest index) minimum wins
                bc = cost;
                bi = c;
            }
        }
        a.best[r] = bi;
    }
}

__global__ __launch_bounds__(256) void pair_count_kernel(PairArgs a)
{
    const int f = blockIdx.x, p = blockIdx.y;
    const int lo = a.bounds[2 * (p * a.F + f)], hi = a.bounds[2 * (p * a.F + f) + 1];
    int c = 0;
    for (int r = lo + threadIdx.x; r < hi; r += blockDim.x) {
        const int j = a.best[r];
        c += (j >= 0 && a.best[j] == r) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    __shared__ int red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) a.cnt[f * a.B + p] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void pair_write_kernel(PairArgs a, ulm_loc3d_t *__restrict__ out,
                                                         int out_capacity)
{
    const int f = blockIdx.x, p = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ int wave_tot[4];
    int base = a.off[f * a.B + p];
    const int lo = a.bounds[2 * (p * a.F + f)], hi = a.bounds[2 * (p * a.F + f) + 1];
    for (int r0 = lo; r0 < hi; r0 += blockDim.x) {
        const int r = r0 + threadIdx.x;
        int j = -1;
        if (r < hi) {
            j = a.best[r];
            if (j >= 0 && a.best[j] != r) j = -1;
        }
        const bool take = j >= 0;
        const unsigned long long bal = __ballot(take);
        if (lane == 0) wave_tot[wv] = __popcll(bal);
        __syncthreads();
        int o = base + __popcll(bal & ((1ull << lane) - 1ull));
        for (int q = 0; q < wv; ++q) o += wave_tot[q];
        if (take && o < out_capacity) {
            const ulm_loc_t xa = a.locs[r], yb = a.locs[j];
            ulm_loc3d_t v;
            v.frame = f;
            v.x = xa.u;
            v.y = yb.u;
            v.z = (xa.z + yb.z) * 0.5f;
            v.i_xz = xa.intensity;
            v.i_yz = yb.intensity;
            v.idx_xz = r;
            v.idx_yz = j;
            out[o] = v;
        }
        base += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
        __syncthreads();
    }
}

hipError_t launch_scan(const int *cnt, int *off, int n, int *count, hipStream_t st);

size_t pair_workspace_bytes(int planes, int F, int capacity) {
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return a256(sizeof(int) * 2 * (size_t)planes * F) + a256(sizeof(int) * (size_t)capacity) +
           2 * a256(sizeof(int) * (size_t)F * (planes / 2));
}

hipError_t launch_pairing(const ulm_ctx *ctx, const ulm_loc_t *locs, const int *count,
                          int capacity, ulm_loc3d_t *out, int out_capacity, int *out_count,
                          char *pws, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int planes = g.n_planes, F = g.n_frames;
    int *bounds = (int *)pws;
    int *best = (int *)(pws + a256(sizeof(int) * 2 * (size_t)planes * F));
    const int B = g.n_blocks;
    int *cnt = (int *)((char *)best + a256(sizeof(int) * (size_t)std::max(capacity, 1)));
    int *off = (int *)((char *)cnt + a256(sizeof(int) * (size_t)F * B));
    const int nkeys = planes * F;
    hipLaunchKernelGGL(pair_bounds_kernel, dim3(cdiv(nkeys, 256)), dim3(256), 0, st, locs, count,
                       capacity, nkeys, F, bounds);
    PairArgs a;
    a.locs = locs;
    a.n = capacity;
    a.F = F;
    a.B = g.n_blocks;
    a.per = cdiv(ctx->cfg.nv, g.n_blocks);
    a.bounds = bounds;
    a.best = best;
    a.cnt = cnt;
    a.off = off;
    hipLaunchKernelGGL(pair_best_kernel, dim3(F, planes), dim3(256), 0, st, a);
    hipLaunchKernelGGL(pair_count_kernel, dim3(F, B), dim3(256), 0, st, a);
    hipError_t e = launch_scan(cnt, off, F * B, out_count, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pair_write_kernel, dim3(F, B), dim3(256), 0, st, a, out, out_capacity);
    return hipGetLastError();
}

}  // namespace ulm
