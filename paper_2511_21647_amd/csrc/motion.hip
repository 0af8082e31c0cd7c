// Rigid motion estimation on the stage-1 reference slices (paper Section
// II-A3): each frame of each of the 2K slices is compared with a reference frame
// by the normalised cross-correlation of the two envelopes, the displacement is
// the sub-pixel peak of that correlation within a lag window, the K
// displacements of each orientation are averaged, and the RC (x-z) and CR (y-z)
// motions are combined into a 3D motion (x from RC, y from CR, the mean of the
// two axial parts).
//
// The paper evaluates the correlation in the Fourier domain (two forward FFTs
// and one inverse per frame).  Only the lags inside the window are needed, and
// the reference is shared by all frames of a slice, so here the correlation is
// one dense contraction per slice:
//   C[f][lag] = sum_p a_f(p) b'(p - lag)        (circular in p)
// with M = frames, N = lags, K = pixels, on v_mfma_f32_32x32x2f32 (FP32 products
// and accumulation, FP64 across work-groups).  a_f = |S_k(f)|, b' = |S_k(ref)|
// minus its mean; the mean of a_f is removed afterwards from the sums of a_f.
//
//   mot_ref_kernel    centred reference envelope b' and its sums (one WG per slice)
//   mot_corr_kernel   partial C over a band of rows for 32 frames, all lags, and
//                     the band's sums of a_f and a_f^2
//   mot_peak_kernel   C and the NCC per (slice, frame), windowed peak (FP32
//                     decisions, first maximum in raster order of the lags),
//                     3-point sub-pixel fit per axis
//   mot_mean_kernel   per-orientation means and the 3D motion per frame
#include "common.h"

#include <math.h>

namespace ulm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMotFrames = 32;     // frames per work-group: the MFMA's M
constexpr int kMotRows = 16;       // slice rows per work-group
constexpr int kMotStage = 256;     // pixels staged in LDS per step
constexpr int kMotAS = kMotStage + 1;
constexpr int kMotMaxLag = 10;     // lag window |dz|, |du| <= L, L <= 10

struct MotArgs {
    int F, nz, nu, npix, K2;       // frames, slice size, 2K slices
    int L, NL;                     // max lag, lags (2L+1)^2
    int nfb, nrc, ref;             // frame blocks, row bands, reference frame
};

__device__ inline double block_sum_1024(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];   // fixed order
    return s;
}

__global__ __launch_bounds__(1024) void mot_ref_kernel(const float2 *__restrict__ S, MotArgs a,
                                                       float *__restrict__ bref,
                                                       double *__restrict__ bstat)
{
    __shared__ double red[16];
    const int s = blockIdx.x;
    const float2 *src = S + ((size_t)s * a.F + a.ref) * a.npix;
    float *dst = bref + (size_t)s * a.npix;
    double acc = 0.0;
    for (int p = threadIdx.x; p < a.npix; p += blockDim.x) {
        const float2 x = src[p];
        acc += (double)sqrtf(x.x * x.x + x.y * x.y);
    }
    const double mu = block_sum_1024(acc, red) / a.npix;
    double s1 = 0.0, s2 = 0.0;
    for (int p = threadIdx.x; p < a.npix; p += blockDim.x) {
        const float2 x = src[p];
        const float v = (float)((double)sqrtf(x.x * x.x + x.y * x.y) - mu);
        dst[p] = v;
        s1 += v;
        s2 += (double)v * v;
    }
    s1 = block_sum_1024(s1, red);
    s2 = block_sum_1024(s2, red);
    if (threadIdx.x == 0) {
        bstat[2 * s] = s1;
        bstat[2 * s + 1] = s2;
    }
}

// LDS: the reference band with a circular halo of L rows and columns, then the
// staged envelopes [32 frames][256 pixels (+1)]; reused for the wave reduction.
size_t mot_corr_lds(int nu, int L, int NT) {
    const size_t tiles = (size_t)(kMotRows + 2 * L) * (nu + 2 * L) + (size_t)kMotFrames * kMotAS;
    const size_t red = (size_t)NT * 32 * 32;
    return sizeof(float) * (tiles > red ? tiles : red);
}

template <int NT>
__global__ __launch_bounds__(256) void mot_corr_kernel(const float2 *__restrict__ S,
                                                       const float *__restrict__ bref, MotArgs a,
                                                       float *__restrict__ part,
                                                       double *__restrict__ astat)
{
    int w = blockIdx.x;
    const int rc = w % a.nrc;
    w /= a.nrc;
    const int fb = w % a.nfb, s = w / a.nfb;
    const int L = a.L, W2 = a.nu + 2 * L, z0 = rc * kMotRows;
    const int rows = min(kMotRows, a.nz - z0);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i32 = lane & 31, hk = lane >> 5;

    extern __shared__ float smem[];
    float *Bs = smem;                                   // [rows + 2L][W2]
    float *As = smem + (size_t)(kMotRows + 2 * L) * W2; // [32][kMotAS]

    const float *bs = bref + (size_t)s * a.npix;
    for (int e = t; e < (rows + 2 * L) * W2; e += 256) {
        const int r = e / W2, c = e % W2;
        int zz = z0 - L + r, uu = c - L;
        zz = zz < 0 ? zz + a.nz : (zz >= a.nz ? zz - a.nz : zz);
        uu = uu < 0 ? uu + a.nu : (uu >= a.nu ? uu - a.nu : uu);
        Bs[e] = bs[(size_t)zz * a.nu + uu];
    }
    // wave w: lag tiles of half w / 2 (NH of the NT tiles), pixels of half w % 2
    // of every staged step; the two waves of a tile half are summed at the end
    constexpr int NH = (NT + 1) / 2;
    const int th = wave >> 1, ph = wave & 1;
    int off[NH];
#pragma unroll
    for (int tt = 0; tt < NH; ++tt) {
        const int j = (th * NH + tt) * 32 + i32;
        off[tt] = 0;
        if (j < a.NL) {
            const int dz = j / (2 * L + 1) - L, du = j % (2 * L + 1) - L;
            off[tt] = dz * W2 + du;
        }
    }
    const int nt_here = min(NH, NT - th * NH);          // tiles of this half (odd NT)
    f32x16 acc[NH];
#pragma unroll
    for (int tt = 0; tt < NH; ++tt) acc[tt] = f32x16{};
    double d1 = 0.0, d2 = 0.0;

    const int npx = rows * a.nu;
    const int f0 = fb * kMotFrames;
    const float2 *Sb = S + (size_t)s * a.F * a.npix + (size_t)z0 * a.nu;
    // the next step's 32 frames of this thread's pixel, in flight during the MFMAs
    float2 xa[kMotFrames];
    auto fetch = [&](int p0n) {
        const int p = p0n + t;
#pragma unroll
        for (int fl = 0; fl < kMotFrames; ++fl) {
            const int f = f0 + fl;
            xa[fl] = (f < a.F && p < npx) ? Sb[(size_t)f * a.npix + p] : make_float2(0.f, 0.f);
        }
    };
    fetch(0);
    for (int p0 = 0; p0 < npx; p0 += kMotStage) {
        __syncthreads();                                // Bs written / previous As consumed
#pragma unroll
        for (int fl = 0; fl < kMotFrames; ++fl)
            As[fl * kMotAS + t] = sqrtf(xa[fl].x * xa[fl].x + xa[fl].y * xa[fl].y);
        __syncthreads();
        if (p0 + kMotStage < npx) fetch(p0 + kMotStage);
        {   // sums of a and a^2 per frame: 8 threads per frame, 32 pixels each
            const int fl = t >> 3, q = t & 7;
            float s1 = 0.f, s2 = 0.f;
            for (int i = 0; i < 32; ++i) {
                const float v = As[fl * kMotAS + q * 32 + i];
                s1 += v;
                s2 = fmaf(v, v, s2);
            }
            for (int o = 1; o < 8; o <<= 1) {
                s1 += __shfl_xor(s1, o);
                s2 += __shfl_xor(s2, o);
            }
            d1 += s1;
            d2 += s2;
        }
        // pixels p0 + 128 ph .. p0 + 128 ph + 127, two per MFMA; (pz, pu) of this
        // lane's pixel advance by two per step (pixels past the band read an
        // in-band reference value and contribute a = 0)
        int pz = (p0 + ph * 128 + hk) / a.nu, pu = (p0 + ph * 128 + hk) - pz * a.nu;
#pragma unroll 2
        for (int st = 0; st < 64; ++st) {
            const int pl = ph * 128 + 2 * st + hk;
            const float av = As[i32 * kMotAS + pl];
            const int base = (min(pz, rows - 1) + L) * W2 + pu + L;
            // every tile slot runs (a slot past the last tile, odd NT only, reads
            // the lag-0 value and is never stored), so the NH reads issue
            // back to back ahead of their MFMAs
            float bv[NH];
#pragma unroll
            for (int tt = 0; tt < NH; ++tt) bv[tt] = Bs[base - off[tt]];
#pragma unroll
            for (int tt = 0; tt < NH; ++tt)
                acc[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[tt], acc[tt], 0, 0, 0);
            pu += 2;
            const bool wrap = pu >= a.nu;
            pu -= wrap ? a.nu : 0;
            pz += wrap ? 1 : 0;
        }
    }
    // sum the two waves of each tile half in a fixed order, in LDS
    float *Red = smem;                                  // [NT][32 frames][32 lags]
    __syncthreads();
    for (int round = 0; round < 2; ++round) {
        if (ph == round) {
#pragma unroll
            for (int tt = 0; tt < NH; ++tt) {
                if (tt >= nt_here) continue;
                const int tg = th * NH + tt;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int r = 8 * (q >> 2) + 4 * hk + (q & 3);
                    float *d = &Red[(tg * 32 + r) * 32 + i32];
                    *d = round == 0 ? acc[tt][q] : *d + acc[tt][q];
                }
            }
        }
        __syncthreads();
    }
    const size_t blk = ((size_t)s * a.nfb + fb) * a.nrc + rc;
    float *dst = part + blk * kMotFrames * (NT * 32);
    for (int e = t; e < kMotFrames * NT * 32; e += 256) {
        const int r = e / (NT * 32), j = e % (NT * 32);
        dst[e] = Red[((j >> 5) * 32 + r) * 32 + (j & 31)];
    }
    if ((t & 7) == 0) {
        double *ds = astat + (blk * kMotFrames + (t >> 3)) * 2;
        ds[0] = d1;
        ds[1] = d2;
    }
}

// 3-point sub-pixel fit (Gaussian, parabolic where a value is <= 0), clamped to
// +-0.5, zero for non-negative curvature.
__device__ inline float mot_fit(float m, float c, float p) {
    float d = 0.f;
    if (m > 0.f && c > 0.f && p > 0.f) {
        const float lm = logf(m), lc = logf(c), lp = logf(p);
        const float den = 2.f * (lm - 2.f * lc + lp);
        if (den < 0.f) d = (lm - lp) / den;
    } else {
        const float den = 2.f * (m - 2.f * c + p);
        if (den < 0.f) d = (m - p) / den;
    }
    return fminf(fmaxf(d, -0.5f), 0.5f);
}

__global__ __launch_bounds__(256) void mot_peak_kernel(const float *__restrict__ part,
                                                       const double *__restrict__ astat,
                                                       const double *__restrict__ bstat, MotArgs a,
                                                       int NTL, float *__restrict__ disp)
{
    __shared__ float ncc[(2 * kMotMaxLag + 1) * (2 * kMotMaxLag + 1)];
    __shared__ float bv[4];
    __shared__ int bi[4];
    const int s = blockIdx.x / a.F, f = blockIdx.x % a.F;
    const int fb = f / kMotFrames, fr = f % kMotFrames;
    const int t = threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int rc = 0; rc < a.nrc; ++rc) {
        const double *st = astat + ((((size_t)s * a.nfb + fb) * a.nrc + rc) * kMotFrames + fr) * 2;
        s1 += st[0];
        s2 += st[1];
    }
    const double N = (double)a.npix;
    const double va = s2 - s1 * s1 / N;
    const double den = va * bstat[2 * s + 1];
    const double mu = s1 / N, sb = bstat[2 * s];
    for (int j = t; j < a.NL; j += 256) {
        double c = 0.0;
        for (int rc = 0; rc < a.nrc; ++rc)
            c += part[((((size_t)s * a.nfb + fb) * a.nrc + rc) * kMotFrames + fr) * NTL + j];
        ncc[j] = den > 0.0 ? (float)((c - mu * sb) / sqrt(den)) : 0.f;
    }
    __syncthreads();
    // first maximum in lag order
    float best = -INFINITY;
    int bj = a.NL;
    for (int j = t; j < a.NL; j += 256) {
        const float v = ncc[j];
        if (v > best) {
            best = v;
            bj = j;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const float ov = __shfl_xor(best, o);
        const int oj = __shfl_xor(bj, o);
        if (ov > best || (ov == best && oj < bj)) {
            best = ov;
            bj = oj;
        }
    }
    if ((t & 63) == 0) {
        bv[t >> 6] = best;
        bi[t >> 6] = bj;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < 4; ++w)
            if (bv[w] > best || (bv[w] == best && bi[w] < bj)) {
                best = bv[w];
                bj = bi[w];
            }
        const int n = 2 * a.L + 1;
        bj = min(bj, a.NL - 1);
        const int iz = bj / n, iu = bj % n;
        float dz = (float)(iz - a.L), du = (float)(iu - a.L);
        if (iz > 0 && iz < n - 1) dz += mot_fit(ncc[bj - n], ncc[bj], ncc[bj + n]);
        if (iu > 0 && iu < n - 1) du += mot_fit(ncc[bj - 1], ncc[bj], ncc[bj + 1]);
        disp[((size_t)s * a.F + f) * 2] = dz;
        disp[((size_t)s * a.F + f) * 2 + 1] = du;
    }
}

__global__ void mot_mean_kernel(const float *__restrict__ disp, int K, int F,
                                float *__restrict__ motion)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double m[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int o = 0; o < 2; ++o)
        for (int k = 0; k < K; ++k)
            for (int c = 0; c < 2; ++c) m[o][c] += disp[(((size_t)o * K + k) * F + f) * 2 + c];
    motion[3 * f] = (float)(m[0][1] / K);
    motion[3 * f + 1] = (float)(m[1][1] / K);
    motion[3 * f + 2] = (float)(0.5 * (m[0][0] / K + m[1][0] / K));
}

struct MotLayout {
    size_t bref, bstat, part, astat, total;
};

static MotLayout mot_layout(const Geometry &g, int L) {
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t K2 = 2 * (size_t)g.n_angles, npix = (size_t)g.nz * g.nu;
    const int NT = cdiv((2 * L + 1) * (2 * L + 1), 32);
    const size_t blocks = K2 * cdiv(g.n_frames, kMotFrames) * cdiv(g.nz, kMotRows);
    MotLayout m;
    size_t off = 0;
    m.bref = off;
    off += a256(sizeof(float) * K2 * npix);
    m.bstat = off;
    off += a256(sizeof(double) * K2 * 2);
    m.part = off;
    off += a256(sizeof(float) * blocks * kMotFrames * NT * 32);
    m.astat = off;
    off += a256(sizeof(double) * blocks * kMotFrames * 2);
    m.total = off;
    return m;
}

size_t motion_workspace_bytes(const Geometry &g, int L) { return mot_layout(g, L).total; }

// LDS bytes of the correlation kernel, or 0 if the plane is too wide for it.
size_t motion_lds_bytes(const Geometry &g, int L) {
    const int NT = cdiv((2 * L + 1) * (2 * L + 1), 32);
    const size_t b = mot_corr_lds(g.nu, L, NT);
    return b <= 150 * 1024 ? b : 0;
}

template <int NT>
static void corr_launch(const float2 *S, const float *bref, const MotArgs &a, float *part,
                        double *astat, size_t lds, hipStream_t st) {
    const int n_wg = a.K2 * a.nfb * a.nrc;
    hipLaunchKernelGGL(mot_corr_kernel<NT>, dim3(n_wg), dim3(256), lds, st, S, bref, a, part, astat);
}

hipError_t launch_motion(const ulm_ctx *ctx, const float2 *S, int ref, int L, float *disp,
                         float *motion, char *mws, hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const MotLayout m = mot_layout(g, L);
    MotArgs a;
    a.F = g.n_frames;
    a.nz = g.nz;
    a.nu = g.nu;
    a.npix = g.nz * g.nu;
    a.K2 = 2 * g.n_angles;
    a.L = L;
    a.NL = (2 * L + 1) * (2 * L + 1);
    a.nfb = cdiv(g.n_frames, kMotFrames);
    a.nrc = cdiv(g.nz, kMotRows);
    a.ref = ref;
    const int NT = cdiv(a.NL, 32);
    float *bref = (float *)(mws + m.bref);
    double *bstat = (double *)(mws + m.bstat);
    float *part = (float *)(mws + m.part);
    double *astat = (double *)(mws + m.astat);
    hipLaunchKernelGGL(mot_ref_kernel, dim3(a.K2), dim3(1024), 0, st, S, a, bref, bstat);
    const size_t lds = mot_corr_lds(g.nu, L, NT);
    switch (NT) {
        case 1: corr_launch<1>(S, bref, a, part, astat, lds, st); break;
        case 2: corr_launch<2>(S, bref, a, part, astat, lds, st); break;
        case 3: corr_launch<3>(S, bref, a, part, astat, lds, st); break;
        case 4: corr_launch<4>(S, bref, a, part, astat, lds, st); break;
        case 6: corr_launch<6>(S, bref, a, part, astat, lds, st); break;
        case 8: corr_launch<8>(S, bref, a, part, astat, lds, st); break;
        case 10: corr_launch<10>(S, bref, a, part, astat, lds, st); break;
        case 12: corr_launch<12>(S, bref, a, part, astat, lds, st); break;
        case 14: corr_launch<14>(S, bref, a, part, astat, lds, st); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mot_peak_kernel, dim3(a.K2 * a.F), dim3(256), 0, st, part, astat, bstat, a,
                       NT * 32, disp);
    hipLaunchKernelGGL(mot_mean_kernel, dim3(cdiv(a.F, 256)), dim3(256), 0, st, disp, g.n_angles,
                       a.F, motion);
    return hipGetLastError();
}

}  // namespace ulm
