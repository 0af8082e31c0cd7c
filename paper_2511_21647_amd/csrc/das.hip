// Stage 1 of the two-stage row-column beamforming (paper Section II-A1): per
// transmit, delay-and-sum of all receive elements into the reference slice
// S_k(u, z).  One work-group owns an 8 x 32 pixel tile, one transmit and 16
// frames: the delay, interpolation weight and phasor of each (pixel, element)
// pair are read once and applied to all 16 frames.  For each element the
// samples that the tile reads (the exact window from the host, staged in
// 16-sample chunks, at most 64 or 128 samples) are staged in LDS,
// double-buffered: the next element's global loads are in flight during the
// current element's arithmetic, so the gathers hit LDS, not the cache.
#include "common.h"

namespace ulm {

// Stage-1 DAS.  The receive part of each (pixel, element) delay and phasor
// comes from host-computed FP64 tables (rounded to FP32):
//   rxd[e][pixel] = (r - z) fs / c,   rxp[e][pixel] = exp(i 2 pi f0 (r - z) / c),
// r = sqrt((u - u_e)^2 + z^2); the per-(depth, transmit) part is
//   (tau_tx + z / c - t_start) fs = sti[k][z] + stz[k][z] (integer + fraction),
//   phz[k][z] = exp(i 2 pi f0 (tau_tx - z / c)).
// The sample index is sti + (rxd + stz): the FP32 sum stays below a few hundred
// samples, and the host forms the same sum to find each (transmit, tile,
// element) window start win[...] exactly.
// LDS holds, per staged sample, (IQ[s], IQ[s+1] - IQ[s]) so the interpolation
// is two FMAs per frame.
// Staging: the window of a (transmit, tile, element) is staged in chunks of 16
// samples x 16 frames, one chunk per wave and step; only the chunks the tile
// reads are staged (the host packs the count beside the window start).  In a
// chunk, lane l stages frame l / 4, run l % 4 (4 samples and their differences),
// so each lane quad loads 17 consecutive samples of one frame.  Which wave
// stages which chunk rotates with the element, so the staging work, and the
// waves that skip it, spread evenly over the SIMDs.
// LDS serves 128 bytes (8 lanes of a 16-byte access) per clock; entry n of
// frame f sits in slot n ^ (2 (f % 2) + (n / 8) % 2), which gives the 8 stores
// of two quads 8 different 16-byte bank groups and keeps consecutive entries
// of a frame in different bank groups for the reads.
__device__ inline int das_slot(int f, int n) { return n ^ ((2 * (f & 1) + ((n >> 3) & 1)) & 3); }
constexpr int kDasChunk = 16;
// window word: start * 16 + (chunks - 1)
__device__ inline int das_lo(int w) { return w >> 4; }
__device__ inline int das_chunks(int w) { return (w & 15) + 1; }

template <int FB, int LEN>
__global__ __launch_bounds__(kDasThreads) void das_stage1_kernel(
    const float2 *__restrict__ iq, float2 *__restrict__ S, const float *__restrict__ stz,
    const int *__restrict__ sti, const float2 *__restrict__ phz, const float *__restrict__ rxd,
    const float2 *__restrict__ rxp, const int *__restrict__ win, Geometry g, int n_tu, int n_tz,
    int n_fb)
{
    const int n_tiles = n_tu * n_tz;
    const int n_wg = n_tiles * n_fb * 2 * g.n_angles;
    const int w = xcd_remap(blockIdx.x, n_wg);
    // tiles fastest: neighbouring tiles of one transmit and frame block share
    // their channel-data windows in L2 (ordering the transmits fastest instead,
    // so that a tile's work-groups share its receive tables, took 18.1 ms
    // instead of 15.8)
    const int tile = w % n_tiles;
    const int fb = (w / n_tiles) % n_fb;
    const int ok = w / (n_tiles * n_fb);
    const int o = ok / g.n_angles, k = ok % g.n_angles;
    const int tz = tile / n_tu, tu = tile % n_tu;

    const int t = threadIdx.x;
    const int iz = tz * kDasTileZ + t / kDasTileU;
    const int iu = tu * kDasTileU + t % kDasTileU;
    const bool valid = iz < g.nz && iu < g.nu;
    const int izc = min(iz, g.nz - 1), iuc = min(iu, g.nu - 1);
    const int npix = g.nz * g.nu;
    const int pix = izc * g.nu + iuc;
    const float stz_p = stz[k * g.nz + izc];
    const int sti_p = sti[k * g.nz + izc];
    const int *wj = win + (size_t)(k * n_tiles + tile) * g.n_elem;

    __shared__ float4 buf[2][FB][LEN];

    const size_t frame_stride = (size_t)2 * g.n_angles * g.n_elem * g.n_samp;
    const int f0 = fb * FB;
    const float2 *blk = iq + ((size_t)o * g.n_angles + k) * g.n_elem * g.n_samp;

    // each wave stages NQ chunks per element: chunk (wave + j + 4 q) % NC
    constexpr int NC = LEN / kDasChunk;
    constexpr int NQ = NC / 4;
    static_assert(kDasThreads == 256 && FB == 16 && NQ >= 1 && NC % 4 == 0, "staging map");
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int sfl = lane >> 2;                 // staged frame
    const int srun = lane & 3;                 // run of 4 samples within the chunk
    // frames past the end read the last frame; their sums are never written
    const float2 *srow = blk + (size_t)min(f0 + sfl, g.n_frames - 1) * frame_stride;
    auto chunk_of = [&](int j, int q) { return (wave + j + 4 * q) & (NC - 1); };
    // two register sets: the global loads of element j + 2 are in flight while
    // element j is applied and element j + 1 (loaded one step earlier) is stored.
    // The loads write their registers unconditionally (start clamped into the
    // record), so nothing waits on them before the store; a chunk that crosses
    // an end of the record is read again, sample by sample with zeros outside,
    // at the store.  A wave whose chunk lies past the window skips both.
    float2 sa[NQ][5], sb[NQ][5];
    auto load = [&](int j, float2 (&st)[NQ][5]) {
        const int wj_ = wj[j];
        const int s_lo = das_lo(wj_), nch = das_chunks(wj_);
        const float2 *row = srow + (size_t)j * g.n_samp;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = chunk_of(j, q);
            if (c < nch) {
                const int gs = max(min(s_lo + kDasChunk * c + 4 * srun, g.n_samp - 5), 0);
#pragma unroll
                for (int i = 0; i < 5; ++i) st[q][i] = row[gs + i];
            }
        }
    };
    // the registers hold the five raw samples until the store, which forms the
    // four (sample, difference) entries
    auto store = [&](int b, int j, int wj_, const float2 (&st)[NQ][5]) {
        const int s_lo = das_lo(wj_), nch = das_chunks(wj_);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = chunk_of(j, q);
            if (c < nch) {
                const int s0 = s_lo + kDasChunk * c;
                const bool inside = s0 >= 0 && s0 + kDasChunk < g.n_samp;
                float2 x[5];
                if (inside) {
#pragma unroll
                    for (int i = 0; i < 5; ++i) x[i] = st[q][i];
                } else {
                    const float2 *row = srow + (size_t)j * g.n_samp;
#pragma unroll
                    for (int i = 0; i < 5; ++i) {
                        const int gi = s0 + 4 * srun + i;
                        const float2 v = row[min(max(gi, 0), g.n_samp - 1)];
                        const bool ok = gi >= 0 && gi < g.n_samp;
                        x[i] = make_float2(ok ? v.x : 0.f, ok ? v.y : 0.f);
                    }
                }
                const int n0 = kDasChunk * c + 4 * srun;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    buf[b][sfl][das_slot(sfl, n0 + i)] =
                        make_float4(x[i].x, x[i].y, x[i + 1].x - x[i].x, x[i + 1].y - x[i].y);
            }
        }
    };

    float2 acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = make_float2(0.f, 0.f);
    auto apply = [&](int cur, float crx, float2 cph, int s_lo) {
        const float s = crx + stz_p;
        const float fl = floorf(s);
        const float fr = s - fl;
        const int idx = min(max((int)fl + sti_p - s_lo, 0), LEN - 1);
        // kAhead LDS reads in flight: frame f + kAhead is requested while frame f
        // is applied
        constexpr int kAhead = 4;
        float4 vq[kAhead];
#pragma unroll
        for (int f = 0; f < kAhead; ++f) vq[f] = buf[cur][f][das_slot(f, idx)];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const float4 v = vq[f % kAhead];
            if (f + kAhead < FB) vq[f % kAhead] = buf[cur][f + kAhead][das_slot(f + kAhead, idx)];
            const float xr = fmaf(fr, v.z, v.x);
            const float xi = fmaf(fr, v.w, v.y);
            acc[f].x = fmaf(cph.x, xr, fmaf(-cph.y, xi, acc[f].x));
            acc[f].y = fmaf(cph.x, xi, fmaf(cph.y, xr, acc[f].y));
        }
        // the sums are complete here: the compiler may not sink this arithmetic
        // past the store's branch (which would keep every LDS read live at once)
#pragma unroll
        for (int f = 0; f < FB; ++f) asm volatile("" : "+v"(acc[f].x), "+v"(acc[f].y));
    };

    const int n = g.n_elem, last = n - 1;
    load(0, sa);
    store(0, 0, wj[0], sa);
    // the receive delay and phasor of the element being applied, and of the next
    float crx = rxd[pix], nrx;
    float2 cph = rxp[pix], nph;
    int s_lo = das_lo(wj[0]);
    load(min(1, last), sb);
    __syncthreads();
    // the last steps re-stage the last element into the idle buffer, so the
    // loop body has no branch around the stores
    for (int j = 0; j < n; j += 2) {
        // buf[0] holds element j, sb element j + 1
        int w_nx = wj[min(j + 1, last)];
        load(min(j + 2, last), sa);
        nrx = rxd[(size_t)min(j + 1, last) * npix + pix];
        nph = rxp[(size_t)min(j + 1, last) * npix + pix];
        apply(0, crx, cph, s_lo);
        store(1, min(j + 1, last), w_nx, sb);
        crx = nrx;
        cph = nph;
        s_lo = das_lo(w_nx);
        __syncthreads();
        if (j + 1 < n) {
            // buf[1] holds element j + 1, sa element j + 2
            w_nx = wj[min(j + 2, last)];
            load(min(j + 3, last), sb);
            nrx = rxd[(size_t)min(j + 2, last) * npix + pix];
            nph = rxp[(size_t)min(j + 2, last) * npix + pix];
            apply(1, crx, cph, s_lo);
            store(0, min(j + 2, last), w_nx, sa);
            crx = nrx;
            cph = nph;
            s_lo = das_lo(w_nx);
            __syncthreads();
        }
    }

    if (!valid) return;
    const float2 ph = phz[k * g.nz + izc];
    float2 *dst = S + ((size_t)(o * g.n_angles + k) * g.n_frames) * npix + (size_t)iz * g.nu + iu;
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        if (f0 + f < g.n_frames) {
            float2 v;
            v.x = acc[f].x * ph.x - acc[f].y * ph.y;
            v.y = acc[f].x * ph.y + acc[f].y * ph.x;
            dst[(size_t)(f0 + f) * npix] = v;
        }
    }
}

template <int FB, int LEN>
static void das_launch(const ulm_ctx *ctx, const float2 *iq, float2 *slices, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const Tables &tb = ctx->tab;
    const int n_tu = cdiv(g.nu, kDasTileU), n_tz = cdiv(g.nz, kDasTileZ);
    const int n_fb = cdiv(g.n_frames, FB);
    const int n_wg = n_tu * n_tz * n_fb * 2 * g.n_angles;
    hipLaunchKernelGGL((das_stage1_kernel<FB, LEN>), dim3(n_wg), dim3(kDasThreads), 0, st, iq,
                       slices, tb.stx, tb.sti, tb.phz, tb.rxd, tb.rxp, tb.win, g, n_tu, n_tz, n_fb);
}

hipError_t launch_stage1(const ulm_ctx *ctx, const float2 *iq, float2 *slices, hipStream_t st)
{
    if (ctx->tab.das_len == 64) das_launch<kDasFrames, 64>(ctx, iq, slices, st);
    else das_launch<kDasFrames, 128>(ctx, iq, slices, st);
    return hipGetLastError();
}

}  // namespace ulm
