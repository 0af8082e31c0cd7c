// MB separation of the filtered planes into flow sub-populations (paper Section
// II-A5): at every pixel, the F-point DFT of the slow-time signal, an ideal
// band-pass mask per subset (up = positive-frequency bins 1..H, down = the
// negative ones, H = (F - 1) / 2, each direction split by |frequency| into S
// contiguous speed ranges), and the inverse DFT of each masked spectrum.
//
// sep_kernel: one work-group per (plane, 8 consecutive pixels).  The frames
// of those pixels are staged in LDS ([frame][pixel], pixels fastest, so the
// global loads and stores are 64-byte rows and the butterflies read
// consecutive banks), transformed by a mixed-radix Stockham FFT (radices 4, 2,
// 3, 5, 7) that ping-pongs between two LDS buffers, and the spectrum is kept in
// registers; each subset then rewrites its masked spectrum to LDS, runs the
// inverse transform and streams the result out.  HBM traffic is one read of
// the planes and one write per subset.
#include "common.h"

#include <math.h>

#include <cmath>
#include <vector>

namespace ulm {

constexpr int kSepPix = 8;                  // pixels per work-group
constexpr int kSepThreads = 256;
constexpr int kSepMaxFrames = 512;
constexpr int kSepMaxPass = 12;
constexpr int kSepMaxSub = 16;              // 2 S subsets, S <= 8
constexpr int kSepRegs = (kSepMaxFrames * kSepPix + kSepThreads - 1) / kSepThreads;

struct SepArgs {
    int F, npix, planes, n_sub, H;
    int n_pass;
    int radix[kSepMaxPass];
    int tw_off[kSepMaxPass];                // offset of each pass's twiddles in the table
    unsigned pmag[kSepMaxPass];             // floor(2^32 / p) + 1 for the pass's p (0 when p = 1)
    int n_tw;                               // twiddle entries (all passes)
    const float2 *twt;                      // [n_tw + 21] twiddles, then the radix roots
    int lo[kSepMaxSub], hi[kSepMaxSub];     // |k| range of each subset
};

__device__ inline float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmulf_conj(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// -i z (forward) or +i z (inverse)
template <bool INV>
__device__ inline float2 mul_mi(float2 z) { return INV ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x); }

// In-place R-point DFT of u, u_out[m] = sum_q u[q] exp(-+2 pi i q m / R).
// Radices 2, 3, 4 and 5 use the usual symmetric forms; 7 the direct sum with
// the roots wr[] (exp(-2 pi i q / 7)).
template <int R, bool INV>
__device__ inline void sep_dft(float2 (&u)[R], const float2 *wr)
{
    auto add = [](float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); };
    auto sub = [](float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); };
    auto scl = [](float2 a, float s) { return make_float2(a.x * s, a.y * s); };
    if constexpr (R == 2) {
        const float2 a = u[0], b = u[1];
        u[0] = add(a, b);
        u[1] = sub(a, b);
    } else if constexpr (R == 4) {
        const float2 s02 = add(u[0], u[2]), d02 = sub(u[0], u[2]);
        const float2 s13 = add(u[1], u[3]), d13 = mul_mi<INV>(sub(u[1], u[3]));
        u[0] = add(s02, s13);
        u[2] = sub(s02, s13);
        u[1] = add(d02, d13);
        u[3] = sub(d02, d13);
    } else if constexpr (R == 3) {
        constexpr float h = 0.866025403784438646763723f;     // sin(2 pi / 3)
        const float2 t1 = add(u[1], u[2]);
        const float2 t2 = sub(u[0], scl(t1, 0.5f));
        const float2 t3 = mul_mi<INV>(scl(sub(u[1], u[2]), h));
        u[0] = add(u[0], t1);
        u[1] = add(t2, t3);
        u[2] = sub(t2, t3);
    } else if constexpr (R == 5) {
        constexpr float c1 = 0.309016994374947424102293f;     // cos(2 pi / 5)
        constexpr float c2 = -0.809016994374947424102293f;    // cos(4 pi / 5)
        constexpr float s1 = 0.951056516295153572116439f;     // sin(2 pi / 5)
        constexpr float s2 = 0.587785252292473129168706f;     // sin(4 pi / 5)
        const float2 t1 = add(u[1], u[4]), t2 = add(u[2], u[3]);
        const float2 t3 = sub(u[1], u[4]), t4 = sub(u[2], u[3]);
        const float2 a1 = add(u[0], add(scl(t1, c1), scl(t2, c2)));
        const float2 a2 = add(u[0], add(scl(t1, c2), scl(t2, c1)));
        const float2 b1 = mul_mi<INV>(add(scl(t3, s1), scl(t4, s2)));
        const float2 b2 = mul_mi<INV>(sub(scl(t3, s2), scl(t4, s1)));
        u[0] = add(u[0], add(t1, t2));
        u[1] = add(a1, b1);
        u[4] = sub(a1, b1);
        u[2] = add(a2, b2);
        u[3] = sub(a2, b2);
    } else {
        float2 o[R];
#pragma unroll
        for (int qo = 0; qo < R; ++qo) {
            float2 acc = u[0];
#pragma unroll
            for (int q = 1; q < R; ++q) {
                const float2 w = wr[(q * qo) % R];
                const float2 t = INV ? cmulf_conj(u[q], w) : cmulf(u[q], w);
                acc.x += t.x;
                acc.y += t.y;
            }
            o[qo] = acc;
        }
#pragma unroll
        for (int qo = 0; qo < R; ++qo) u[qo] = o[qo];
    }
}

// One Stockham pass of radix R over every pixel: x -> y.  p = product of the
// radices of the earlier passes; tw[k R + q] = exp(-2 pi i q k / (p R)) for
// k < p; wr[q] = exp(-2 pi i q / R).  INV uses the conjugates.  i mod p comes
// from a multiply-high by pmag = floor(2^32 / p) + 1, exact for i, p < 2^16.
template <int R, bool INV>
__device__ void sep_pass(const float2 *__restrict__ x, float2 *__restrict__ y, int F, int p,
                         unsigned pmag, const float2 *tw, const float2 *wr)
{
    const int nb = F / R;                                  // butterflies per pixel
    for (int e = threadIdx.x; e < nb * kSepPix; e += kSepThreads) {
        const int i = e / kSepPix, px = e % kSepPix;
        const int k = p == 1 ? 0 : i - (int)__umulhi((unsigned)i, pmag) * p;
        float2 u[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 v = x[(i + q * nb) * kSepPix + px];
            if (q > 0) v = INV ? cmulf_conj(v, tw[k * R + q]) : cmulf(v, tw[k * R + q]);
            u[q] = v;
        }
        const int j = (i - k) * R + k;
        sep_dft<R, INV>(u, wr);
#pragma unroll
        for (int qo = 0; qo < R; ++qo) y[(j + qo * p) * kSepPix + px] = u[qo];
    }
}

// All passes; returns the buffer that holds the result.
template <bool INV>
__device__ float2 *sep_fft(float2 *a, float2 *b, const SepArgs &g, const float2 *tw,
                           const float2 *wr)
{
    int p = 1;
    for (int s = 0; s < g.n_pass; ++s) {
        const int R = g.radix[s];
        const float2 *t = tw + g.tw_off[s];
        switch (R) {
            case 2: sep_pass<2, INV>(a, b, g.F, p, g.pmag[s], t, wr + 0); break;
            case 3: sep_pass<3, INV>(a, b, g.F, p, g.pmag[s], t, wr + 2); break;
            case 4: sep_pass<4, INV>(a, b, g.F, p, g.pmag[s], t, wr + 5); break;
            case 5: sep_pass<5, INV>(a, b, g.F, p, g.pmag[s], t, wr + 9); break;
            default: sep_pass<7, INV>(a, b, g.F, p, g.pmag[s], t, wr + 14); break;
        }
        __syncthreads();
        float2 *c = a;
        a = b;
        b = c;
        p *= R;
    }
    return a;
}

__global__ __launch_bounds__(kSepThreads) void sep_kernel(const float2 *__restrict__ P,
                                                          float2 *__restrict__ out, SepArgs g)
{
    extern __shared__ float2 sm[];
    float2 *buf0 = sm;                                     // [F][kSepPix]
    float2 *buf1 = sm + (size_t)g.F * kSepPix;
    float2 *tw = buf1 + (size_t)g.F * kSepPix;             // [n_tw]
    float2 *wr = tw + g.n_tw;                              // radix roots: 2, 3, 4, 5, 7 -> 21
    const int groups = cdiv(g.npix, kSepPix);
    const int plane = blockIdx.x / groups, px0 = (blockIdx.x % groups) * kSepPix;
    const int t = threadIdx.x;

    // twiddles of every pass and the roots of unity of every radix, from the
    // context's table (tw and wr are contiguous, as in the table)
    for (int e = t; e < g.n_tw + 21; e += kSepThreads) tw[e] = g.twt[e];
    const float2 *src = P + (size_t)plane * g.F * g.npix + px0;
    const int npx = min(kSepPix, g.npix - px0);
    for (int e = t; e < g.F * kSepPix; e += kSepThreads) {
        const int f = e / kSepPix, px = e % kSepPix;
        buf0[e] = px < npx ? src[(size_t)f * g.npix + px] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const float2 *X = sep_fft<false>(buf0, buf1, g, tw, wr);
    // the spectrum stays in registers: element e = t + 256 r
    float2 xr[kSepRegs];
    int nreg = 0;
#pragma unroll
    for (int r = 0; r < kSepRegs; ++r) {
        const int e = t + r * kSepThreads;
        if (e < g.F * kSepPix) {
            xr[r] = X[e];
            nreg = r + 1;
        }
    }
    const float scale = 1.0f / (float)g.F;
    const size_t sub_stride = (size_t)g.planes * g.F * g.npix;
    for (int s = 0; s < g.n_sub; ++s) {
        const bool up = s < g.n_sub / 2;
        const int lo = g.lo[s], hi = g.hi[s];
        __syncthreads();                                    // previous subset's reads done
#pragma unroll
        for (int r = 0; r < kSepRegs; ++r) {
            if (r < nreg) {
                const int e = t + r * kSepThreads;
                if (e < g.F * kSepPix) {
                    const int k = e / kSepPix;
                    const int m = up ? k : g.F - k;
                    const bool keep = (up ? (k >= 1 && k <= g.H) : (k >= g.F - g.H)) && m >= lo && m < hi;
                    buf0[e] = keep ? xr[r] : make_float2(0.f, 0.f);
                }
            }
        }
        __syncthreads();
        const float2 *Y = sep_fft<true>(buf0, buf1, g, tw, wr);
        float2 *dst = out + s * sub_stride + (size_t)plane * g.F * g.npix + px0;
        for (int e = t; e < g.F * kSepPix; e += kSepThreads) {
            const int f = e / kSepPix, px = e % kSepPix;
            if (px < npx) {
                const float2 v = Y[e];
                dst[(size_t)f * g.npix + px] = make_float2(v.x * scale, v.y * scale);
            }
        }
    }
}

// Radices for F (4 first, then 2, 3, 5, 7); false if F has another prime factor.
static bool sep_factor(int F, SepArgs &g) {
    g.n_pass = 0;
    int n = F, off = 0, p = 1;
    const int order[5] = {4, 2, 3, 5, 7};
    for (int r : order) {
        while (n % r == 0) {
            if (g.n_pass == kSepMaxPass) return false;
            g.radix[g.n_pass] = r;
            g.tw_off[g.n_pass] = off;
            g.pmag[g.n_pass] = p == 1 ? 0u : (unsigned)((1ull << 32) / (unsigned)p + 1ull);
            off += p * r;
            p *= r;
            ++g.n_pass;
            n /= r;
        }
    }
    g.n_tw = off;
    return n == 1;
}

bool separate_supported(int F) {
    SepArgs g;
    return F >= 2 && F <= kSepMaxFrames && sep_factor(F, g);
}

// The kernel's table for F frames: tw[tw_off[s] + k R + q] = exp(-2 pi i q k /
// (p R)) for every pass s (radix R, p = product of the earlier radices), then
// the roots exp(-2 pi i q / R) of R = 2, 3, 4, 5, 7 (2 + 3 + 4 + 5 + 7 = 21
// entries); FP64, rounded to FP32.  Empty if F is not supported.
std::vector<float2> separate_twiddles(int F) {
    SepArgs g;
    if (!separate_supported(F)) return {};
    sep_factor(F, g);
    std::vector<float2> t((size_t)g.n_tw + 21);
    auto root = [](double turns) {      // exp(2 pi i turns)
        return make_float2((float)std::cos(2.0 * M_PI * turns), (float)std::sin(2.0 * M_PI * turns));
    };
    int p = 1;
    for (int s = 0; s < g.n_pass; ++s) {
        const int R = g.radix[s];
        for (int e = 0; e < p * R; ++e) {
            const int k = e / R, q = e % R;
            t[g.tw_off[s] + e] = root(-(double)((long)q * k % (p * R)) / (double)(p * R));
        }
        p *= R;
    }
    const int rad[5] = {2, 3, 4, 5, 7};
    int o = g.n_tw;
    for (int r : rad)
        for (int q = 0; q < r; ++q) t[o++] = root(-(double)q / (double)r);
    return t;
}

size_t separate_lds_bytes(int F) {
    SepArgs g;
    sep_factor(F, g);
    return sizeof(float2) * ((size_t)2 * F * kSepPix + g.n_tw + 21);
}

hipError_t launch_separate(const ulm_ctx *ctx, const float2 *P, int n_speed, float2 *out,
                           hipStream_t st)
{
    const Geometry &geo = ctx->geo;
    SepArgs g;
    if (!sep_factor(geo.n_frames, g)) return hipErrorInvalidValue;
    g.F = geo.n_frames;
    g.npix = geo.nz * geo.nu;
    g.planes = geo.n_planes;
    g.n_sub = 2 * n_speed;
    g.H = (g.F - 1) / 2;
    for (int d = 0; d < 2; ++d)
        for (int s = 0; s < n_speed; ++s) {
            g.lo[d * n_speed + s] = 1 + (s * g.H) / n_speed;
            g.hi[d * n_speed + s] = 1 + ((s + 1) * g.H) / n_speed;
        }
    g.twt = ctx->tab.sep_tw;
    if (!g.twt) return hipErrorInvalidValue;
    const int groups = cdiv(g.npix, kSepPix);
    hipLaunchKernelGGL(sep_kernel, dim3(groups * g.planes), dim3(kSepThreads),
                       separate_lds_bytes(g.F), st, P, out, g);
    return hipGetLastError();
}

}  // namespace ulm
