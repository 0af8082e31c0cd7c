// Eigen-based SVD clutter filter (paper Section II-A2) of each projection
// plane's Casorati matrix I (pixels x frames):
//   1. covariance C = I^H I   (gram_f64_kernel + gram_reduce_kernel, FP64 MFMA;
//      gram_bf16x3_kernel for the split-precision form)
//   2. eigendecomposition of C in FP64 (eigen_kernel: Householder
//      tridiagonalisation, bisection on Sturm counts, inverse iteration for the
//      clutter eigenvectors, back-transformation)
//   3. removal I_f = I - (I V_c) V_c^H   (removal_f64_kernel, FP64 MFMA;
//      removal_bf16_kernel for the split-precision form)
// Layout: a plane is stored frame-major, [F][n_pix] complex64, i.e. the
// transpose of the Casorati matrix; the frame axis is the Gram's output axis
// and the pixel axis its reduction axis.
#include "eigen.h"

#include <float.h>
#include <stdlib.h>

namespace ulm {


typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ inline void pair_of(int pair, int nblk, int &I, int &J) {
    int p = pair;
    for (I = 0; I < nblk; ++I) {
        const int n = nblk - I;
        if (p < n) { J = I + p; return; }
        p -= n;
    }
    I = J = 0;
}

// ---------------------------------------------------------------- Gram, FP64 MFMA
// One work-group: one plane, one 64x64 block pair (I <= J) of C, one chunk of
// pixels.  Four waves, each a 32x32 quadrant = 2x2 tiles of
// v_mfma_f64_16x16x4f64.  K = 4 per instruction = 2 pixels x (re, im):
//   C_re += A . B      with A[f][k], B[k][f'] = (re, im) of pixel p
//   C_im += A . B'     with B'[k][f'] = (im, -re)
// FP32 inputs are exact in FP64, so every product is exact and only FP64
// summation rounds.
__global__ __launch_bounds__(256) void gram_f64_kernel(const float2 *__restrict__ P,
                                                       double2 *__restrict__ part, int F,
                                                       int npix, int pairs, int chunks, int nblk)
{
    // the block pairs of one pixel chunk run back to back on one XCD, so the
    // frame blocks they share are read from that XCD's L2
    const int wl = xcd_remap(blockIdx.x, gridDim.x);
    const int pair = wl % pairs;
    const int chunk = (wl / pairs) % chunks;
    const int plane = wl / (chunks * pairs);
    int I, J;
    pair_of(pair, nblk, I, J);
    const float2 *src = P + (size_t)plane * F * npix;
    const int px0 = chunk * kGramChunk;
    const int px1 = min(px0 + kGramChunk, npix);

    __shared__ float2 lds[2 * kGramBlock][kGramStage + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    // in a diagonal block the lower-left quadrant mirrors the upper-right one
    // (C is Hermitian, and the reduction reads it from there): its wave only
    // stages pixels
    const bool mirror = I == J && wi == 1 && wj == 0;
    const int kk = lane >> 4, r16 = lane & 15;

    f64x4 accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accr[a][b] = f64x4{0, 0, 0, 0};
            acci[a][b] = f64x4{0, 0, 0, 0};
        }

    // the next stage's pixels are loaded into registers while this stage's
    // products run
    constexpr int kPer = 2 * kGramBlock * kGramStage / 256;
    float2 pre[kPer];
    auto fetch = [&](int p0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int row = e / kGramStage, col = e % kGramStage;
            const int frame = row < kGramBlock ? I * kGramBlock + row : J * kGramBlock + row - kGramBlock;
            const int px = p0 + col;
            pre[i] = make_float2(0.f, 0.f);
            if (frame < F && px < px1) pre[i] = src[(size_t)frame * npix + px];
        }
    };
    fetch(px0);
    for (int p0 = px0; p0 < px1; p0 += kGramStage) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            lds[e / kGramStage][e % kGramStage] = pre[i];
        }
        __syncthreads();
        if (p0 + kGramStage < px1) fetch(p0 + kGramStage);
        // the mirror wave of a diagonal block forms nothing; the others' 16
        // steps are unrolled whole (a static trip count)
        if (!mirror)
#pragma unroll
        for (int step = 0; step < kGramStage / 2; ++step) {
            const int pxl = step * 2 + (kk >> 1);
            const bool im = kk & 1;
            double a[2], br[2], bi[2];
#pragma unroll
            for (int ti = 0; ti < 2; ++ti) {
                const float2 v = lds[wi * 32 + ti * 16 + r16][pxl];
                a[ti] = im ? v.y : v.x;
            }
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) {
                const float2 v = lds[kGramBlock + wj * 32 + tj * 16 + r16][pxl];
                br[tj] = im ? v.y : v.x;
                bi[tj] = im ? -v.x : v.y;
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    accr[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], br[tj], accr[ti][tj], 0, 0, 0);
                    acci[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], bi[tj], acci[ti][tj], 0, 0, 0);
                }
        }
        __syncthreads();
    }

    double2 *dst = part + ((size_t)(plane * pairs + pair) * chunks + chunk) * kGramBlock * kGramBlock;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // v_mfma_f64_16x16x4f64 result: lane l, register r holds D[4 r + l / 16][l % 16]
                const int row = wi * 32 + ti * 16 + 4 * r + kk;
                const int col = wj * 32 + tj * 16 + r16;
                dst[row * kGramBlock + col] = make_double2(accr[ti][tj][r], acci[ti][tj][r]);
            }
}

// Three-term BF16 split of a value (hi, mid, lo).
struct bf16x3 { __bf16 h, m, l; };

__device__ inline bf16x3 split3(float x) {
    bf16x3 o;
    o.h = (__bf16)x;
    float r = x - (float)o.h;      // exact
    o.m = (__bf16)r;
    r -= (float)o.m;               // exact
    o.l = (__bf16)r;
    return o;
}

__device__ inline bf16x3 split3(double x) {
    bf16x3 o;
    o.h = (__bf16)(float)x;
    double r = x - (double)(float)o.h;
    o.m = (__bf16)(float)r;
    r -= (double)(float)o.m;
    o.l = (__bf16)(float)r;
    return o;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
struct bf16x2x3 { bf16x2 h, m, l; };

// Three-term split of two floats at once (one packed conversion per term).
__device__ inline bf16x2x3 split3x2(f32x2 x) {
    bf16x2x3 o;
    o.h = __builtin_convertvector(x, bf16x2);
    f32x2 r = x - __builtin_convertvector(o.h, f32x2);     // exact
    o.m = __builtin_convertvector(r, bf16x2);
    r -= __builtin_convertvector(o.m, f32x2);              // exact
    o.l = __builtin_convertvector(r, bf16x2);
    return o;
}

__device__ inline bf16x8 cat4(bf16x2 a, bf16x2 b, bf16x2 c, bf16x2 d) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const bf16x4 ab = __builtin_shufflevector(a, b, 0, 1, 2, 3);
    const bf16x4 cd = __builtin_shufflevector(c, d, 0, 1, 2, 3);
    return __builtin_shufflevector(ab, cd, 0, 1, 2, 3, 4, 5, 6, 7);
}

// element j of the three term vectors t[0..2] <- the terms of x
#define ULM_SET3(t, j, x)        \
    do {                         \
        const bf16x3 s3_ = split3(x); \
        (t)[0][j] = s3_.h;       \
        (t)[1][j] = s3_.m;       \
        (t)[2][j] = s3_.l;       \
    } while (0)

// ---------------------------------------------------------------- Gram, BF16 split
// Split-precision form: every value is a sum of kSplitTerms = 3 BF16 terms,
// x = hi + mid + lo (hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi -
// mid): exact for FP32 data), and the products of terms whose orders add up
// to less than three (hi.hi, hi.mid, mid.hi, hi.lo, mid.mid, lo.hi) run on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  (Two terms with hi.hi +
// hi.lo + lo.hi leave a relative error of 2^-17 per product; where the
// clutter eigenvalues span four decades that moves the filtered planes by
// about 1e-3.)  The complex Gram is formed from real products of the real and
// imaginary planes: with a = row f1, b = row f2 of the stack,
//   C_re = a_re . b_re + a_im . b_im,   C_im = a_re . b_im - a_im . b_re,
// K = 16 pixels per instruction.  Each element is split once, when the
// work-group stages it: a thread loads eight consecutive pixels of a frame
// (prefetched one stage ahead), splits them and writes six 16-byte BF16 rows
// (re hi, mid, lo, im hi, mid, lo) to LDS, which is double-buffered, so a
// stage needs one barrier and its inner loop only reads LDS and issues MFMAs.
// The imaginary part takes a_im with its sign bits flipped, so a stage has two
// FP32 accumulators, which are added into FP64 after every stage: the FP32
// rounding then applies to 16-pixel partial sums only, not to the running
// covariance (an FP32 running sum would leave a relative error near 1e-7 in
// C and, amplified by the eigenvalue spread, about 1e-4 in the filtered
// planes).  One wave per 32x32 quadrant of the 64x64 block pair.
constexpr int kG16Stage = 16;                    // pixels per stage (one K-step)
constexpr int kG16Pitch = kG16Stage + 8;         // BF16 per LDS row (padded against bank conflicts)
constexpr int kG16Rows = 2 * kGramBlock;         // frames of the two blocks

__global__ __launch_bounds__(256, 2) void gram_bf16x3_kernel(const float2 *__restrict__ P,
                                                             double2 *__restrict__ part, int F,
                                                             int npix, int pairs, int chunks,
                                                             int nblk)
{
    constexpr int NT = kSplitTerms;
    // block pairs of one pixel chunk back to back on one XCD (shared frame blocks in its L2)
    const int wl = xcd_remap(blockIdx.x, gridDim.x);
    const int pair = wl % pairs;
    const int chunk = (wl / pairs) % chunks;
    const int plane = wl / (chunks * pairs);
    int I, J;
    pair_of(pair, nblk, I, J);
    const float2 *src = P + (size_t)plane * F * npix;
    const int px0 = chunk * kGramChunk;
    const int px1 = min(px0 + kGramChunk, npix);

    // [buffer][re terms 0..NT-1, im terms 0..NT-1][row][pixel]
    __shared__ __attribute__((aligned(16))) __bf16 lds[2][2 * NT][kG16Rows][kG16Pitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int half = lane >> 5, r32 = lane & 31;

    // staging: thread t owns pixels (t % 2) * 8 .. + 7 of row t / 2
    const int sg = threadIdx.x & 1, srow = threadIdx.x >> 1;
    const int sframe = srow < kGramBlock ? I * kGramBlock + srow : J * kGramBlock + srow - kGramBlock;
    const float2 *srcrow = src + (size_t)min(sframe, F - 1) * npix;
    float2 pre[8];
    auto fetch = [&](int p0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int px = p0 + sg * 8 + q;
            const float2 v = srcrow[min(px, px1 - 1)];
            pre[q] = (sframe < F && px < px1) ? v : make_float2(0.f, 0.f);
        }
    };
    auto stage = [&](int buf) {
        // pixels 2p, 2p + 1 split together
        bf16x2x3 re[4], im[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            re[p] = split3x2(f32x2{pre[2 * p].x, pre[2 * p + 1].x});
            im[p] = split3x2(f32x2{pre[2 * p].y, pre[2 * p + 1].y});
        }
        bf16x8 *row = reinterpret_cast<bf16x8 *>(&lds[buf][0][srow][sg * 8]);
        constexpr int kPlane = kG16Rows * kG16Pitch / 8;       // bf16x8 per term plane
        row[0 * kPlane] = cat4(re[0].h, re[1].h, re[2].h, re[3].h);
        row[1 * kPlane] = cat4(re[0].m, re[1].m, re[2].m, re[3].m);
        row[2 * kPlane] = cat4(re[0].l, re[1].l, re[2].l, re[3].l);
        row[3 * kPlane] = cat4(im[0].h, im[1].h, im[2].h, im[3].h);
        row[4 * kPlane] = cat4(im[0].m, im[1].m, im[2].m, im[3].m);
        row[5 * kPlane] = cat4(im[0].l, im[1].l, im[2].l, im[3].l);
    };

    double dr[16], di[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) dr[q] = di[q] = 0.0;
    // two sets of FP32 accumulators: a stage's products go to one set while the
    // other set (the previous stage's) is added into FP64, so the additions
    // wait on no MFMA in flight.  The loop body has no branch, so the compiler
    // interleaves the staging of the next pixels with the MFMAs.  (In a diagonal
    // block the lower-left quadrant's wave computes the mirror of the
    // upper-right one, which the reduction does not read.)
    f32x16 s0re = {}, s0im = {}, s1re = {}, s1im = {};

    const int arow = wi * 32 + r32, brow = kGramBlock + wj * 32 + r32;
    const int col = half * 8;
    auto products = [&](int b, f32x16 &c_re, f32x16 &c_im) {
        bf16x8 ar[NT], ai[NT], br[NT], bi[NT], nai[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            ar[k] = *reinterpret_cast<const bf16x8 *>(&lds[b][k][arow][col]);
            ai[k] = *reinterpret_cast<const bf16x8 *>(&lds[b][NT + k][arow][col]);
            br[k] = *reinterpret_cast<const bf16x8 *>(&lds[b][k][brow][col]);
            bi[k] = *reinterpret_cast<const bf16x8 *>(&lds[b][NT + k][brow][col]);
            // -a_im: the sign bits flipped
            u32x4 bits = __builtin_bit_cast(u32x4, ai[k]);
            bits ^= 0x80008000u;
            nai[k] = __builtin_bit_cast(bf16x8, bits);
        }
        // smallest products first, hi.hi last: the FP32 partial sums stay small
        // until the last two instructions, so most roundings are relative to
        // small values
#pragma unroll
        for (int ord = NT - 1; ord >= 0; --ord)
#pragma unroll
            for (int ta = 0; ta <= ord; ++ta) {
                const int tb = ord - ta;
                c_re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ta], br[tb], c_re, 0, 0, 0);
                c_re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[ta], bi[tb], c_re, 0, 0, 0);
                c_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ta], bi[tb], c_im, 0, 0, 0);
                c_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nai[ta], br[tb], c_im, 0, 0, 0);
            }
    };
    // the 16 pixels' sums, rounded in FP32, are added in FP64
    auto fold = [&](f32x16 &c_re, f32x16 &c_im) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            dr[q] += (double)c_re[q];
            di[q] += (double)c_im[q];
        }
        c_re = f32x16{};
        c_im = f32x16{};
    };

    fetch(px0);
    stage(0);
    __syncthreads();
    // stages n (buffer 0, set 0) and n + 1 (buffer 1, set 1) per iteration;
    // past the chunk's end the staged pixels are zeros, so an odd stage count
    // runs one stage of zeros
    for (int p0 = px0; p0 < px1; p0 += 2 * kG16Stage) {
        fetch(p0 + kG16Stage);
        products(0, s0re, s0im);
        fold(s1re, s1im);
        stage(1);
        __syncthreads();
        fetch(p0 + 2 * kG16Stage);
        products(1, s1re, s1im);
        fold(s0re, s0im);
        stage(0);
        __syncthreads();
    }
    fold(s1re, s1im);

    double2 *dst = part + ((size_t)(plane * pairs + pair) * chunks + chunk) * kGramBlock * kGramBlock;
    // 32x32 output layout: acc q -> row 8*(q/4) + 4*half + q%4, column r32
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = wi * 32 + 8 * (q >> 2) + 4 * half + (q & 3);
        const int cc = wj * 32 + r32;
        dst[row * kGramBlock + cc] = make_double2(dr[q], di[q]);
    }
}

// Sum of the per-chunk partials of C.  One work-group per (plane, block pair
// I <= J, 4 rows of the 64 x 64 block): thread (row, column) adds its element
// over the pixel chunks in chunk order, so a row of 64 partials is one
// contiguous read, and writes it to C with its mirror: the conjugate into
// block (J, I), and in a diagonal block the upper-right quadrant's conjugate
// into the lower-left one (whose partials the Gram kernels do not form).
constexpr int kReduceRows = 4;
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double2 *__restrict__ part,
                                                          double2 *__restrict__ C, int F, int pairs,
                                                          int chunks, int nblk)
{
    constexpr int kStrips = kGramBlock / kReduceRows;
    const int strip = blockIdx.x % kStrips;
    const int pair = (blockIdx.x / kStrips) % pairs;
    const int plane = blockIdx.x / (kStrips * pairs);
    int I, J;
    pair_of(pair, nblk, I, J);
    const int r = strip * kReduceRows + (threadIdx.x >> 6), c = threadIdx.x & 63;
    const bool diag = I == J;
    if (diag && r >= kGramBlock / 2 && c < kGramBlock / 2) return;
    const int f1 = I * kGramBlock + r, f2 = J * kGramBlock + c;
    if (f1 >= F || f2 >= F) return;
    const double2 *src = part + (size_t)(plane * pairs + pair) * chunks * kGramBlock * kGramBlock +
                         r * kGramBlock + c;
    double re = 0.0, im = 0.0;
#pragma unroll 8
    for (int ch = 0; ch < chunks; ++ch) {
        const double2 v = src[(size_t)ch * kGramBlock * kGramBlock];
        re += v.x;
        im += v.y;
    }
    double2 *Cp = C + (size_t)plane * F * F;
    Cp[(size_t)f1 * F + f2] = make_double2(re, im);
    if (!diag || (r < kGramBlock / 2 && c >= kGramBlock / 2)) Cp[(size_t)f2 * F + f1] = make_double2(re, -im);
}

// ---------------------------------------------------------------- eigensolver
constexpr int kEigThreads = 512;
constexpr int kEigWaves = kEigThreads / 64;
constexpr int kMaxF = 1024;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kEigWaves; ++i) s += red[i];
    return s;
}

__device__ inline double block_max(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < kEigWaves; ++i) s = fmax(s, red[i]);
    return s;
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconjmul(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Number of eigenvalues of the symmetric tridiagonal (d, e2 = e^2) below x.
__device__ inline int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
        if (fabs(q) <= pivmin) q = -pivmin;
        q = d[i] - x - e2[i - 1] / q;
        cnt += q < 0.0;
    }
    return cnt;
}

// One work-group per plane.  Workspace per plane: C (tridiagonalised in place,
// Householder vectors in the rows), tau, d, e, eigenvalues, and scratch for
// the c tridiagonal eigenvectors (real) and their complex back-transforms.
__global__ __launch_bounds__(kEigThreads) void eigen_kernel(
    double2 *__restrict__ Cbuf, double2 *__restrict__ taubuf, double *__restrict__ dbuf,
    double *__restrict__ ebuf, double *__restrict__ evals, double2 *__restrict__ evecs,
    double *__restrict__ tscratch, double2 *__restrict__ xscratch, int F, int c,
    int *__restrict__ status, double *__restrict__ evals_out, int *__restrict__ eflag)
{
    const int plane = blockIdx.x;
    const int t = threadIdx.x;
    double2 *A = Cbuf + (size_t)plane * F * F;
    double2 *tau = taubuf + (size_t)plane * F;
    double *d = dbuf + (size_t)plane * F;
    double *e = ebuf + (size_t)plane * F;
    double *lam = evals + (size_t)plane * F;
    double2 *V = evecs + (size_t)plane * F * (c > 0 ? c : 1);

    __shared__ double2 sv[kMaxF];
    __shared__ double2 sw[kMaxF];
    __shared__ double2 part[kEigThreads];
    __shared__ double red[kEigWaves];
    __shared__ double sd[kMaxF];
    __shared__ double se2[kMaxF];

    // non-finite covariance: leave the plane unfiltered
    double bad = 0.0;
    for (size_t i = t; i < (size_t)F * F; i += kEigThreads) {
        const double2 v = A[i];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1.0;
    }
    bad = block_max(bad, red);
    if (bad > 0.0) {
        for (int i = t; i < F * c; i += kEigThreads) V[i] = make_double2(0.0, 0.0);
        for (int i = t; i < F; i += kEigThreads) {
            lam[i] = __builtin_nan("");
            if (evals_out) evals_out[(size_t)plane * F + i] = lam[i];
        }
        if (t == 0) {
            atomicOr(status, kStatusNumeric);
            atomicOr(eflag + plane, 1);
        }
        return;
    }

    // 1. Householder reduction to real tridiagonal form, T = Q^H C Q.
    for (int k = 0; k + 1 < F; ++k) {
        const int m = F - k - 1;
        double2 *row = A + (size_t)k * F + k + 1;          // conj of the column below the diagonal
        double nrm = 0.0;
        for (int i = t; i < m; i += kEigThreads) {
            const double2 x = make_double2(row[i].x, -row[i].y);
            sv[i] = x;
            if (i > 0) nrm += x.x * x.x + x.y * x.y;
        }
        nrm = block_sum(nrm, red);
        const double2 alpha = sv[0];
        double2 tk = make_double2(0.0, 0.0);
        double beta = alpha.x;
        if (nrm > 0.0 || alpha.y != 0.0) {
            beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + nrm), alpha.x);
            tk = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            // scale = 1 / (alpha - beta)
            const double2 den = make_double2(alpha.x - beta, alpha.y);
            const double dd = den.x * den.x + den.y * den.y;
            const double2 scale = make_double2(den.x / dd, -den.y / dd);
            __syncthreads();
            for (int i = t; i < m; i += kEigThreads) sv[i] = i == 0 ? make_double2(1.0, 0.0) : cmul(sv[i], scale);
        } else {
            __syncthreads();
            for (int i = t; i < m; i += kEigThreads) sv[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        for (int i = t; i < m; i += kEigThreads) row[i] = sv[i];
        if (t == 0) {
            d[k] = A[(size_t)k * F + k].x;
            e[k] = beta;
            tau[k] = tk;
        }
        if (tk.x == 0.0 && tk.y == 0.0) { __syncthreads(); continue; }

        // p = tau * A22 v, using A22[i][j] = conj(A22[j][i]) for coalesced rows
        double2 *A22 = A + (size_t)(k + 1) * F + (k + 1);
        const int mp = (m + 63) & ~63;
        if (mp <= kEigThreads) {
            const int G = kEigThreads / mp;
            const int i = t % mp, gi = t / mp;
            double2 acc = make_double2(0.0, 0.0);
            if (i < m && gi < G)
                for (int j = gi; j < m; j += G) {
                    const double2 a = A22[(size_t)j * F + i];
                    const double2 v = sv[j];
                    acc.x += a.x * v.x + a.y * v.y;
                    acc.y += a.x * v.y - a.y * v.x;
                }
            part[t] = acc;
            __syncthreads();
            if (t < m) {
                double2 s = make_double2(0.0, 0.0);
                for (int q = 0; q < G; ++q) { s.x += part[q * mp + t].x; s.y += part[q * mp + t].y; }
                sw[t] = cmul(tk, s);
            }
        } else {
            for (int i = t; i < m; i += kEigThreads) {
                double2 acc = make_double2(0.0, 0.0);
                for (int j = 0; j < m; ++j) {
                    const double2 a = A22[(size_t)j * F + i];
                    const double2 v = sv[j];
                    acc.x += a.x * v.x + a.y * v.y;
                    acc.y += a.x * v.y - a.y * v.x;
                }
                sw[i] = cmul(tk, acc);
            }
        }
        __syncthreads();
        // alpha2 = -1/2 tau (p^H v);  w = p + alpha2 v
        double pr = 0.0, pi = 0.0;
        for (int i = t; i < m; i += kEigThreads) {
            const double2 q = cconjmul(sw[i], sv[i]);
            pr += q.x;
            pi += q.y;
        }
        pr = block_sum(pr, red);
        pi = block_sum(pi, red);
        const double2 a2 = cmul(make_double2(-0.5 * tk.x, -0.5 * tk.y), make_double2(pr, pi));
        for (int i = t; i < m; i += kEigThreads) {
            const double2 av = cmul(a2, sv[i]);
            sw[i] = make_double2(sw[i].x + av.x, sw[i].y + av.y);
        }
        __syncthreads();
        // A22 -= v w^H + w v^H
        if (mp <= kEigThreads) {
            const int G = kEigThreads / mp;
            const int j = t % mp, gi = t / mp;
            if (j < m && gi < G) {
                const double2 vj = sv[j], wj = sw[j];
                for (int i = gi; i < m; i += G) {
                    const double2 vi = sv[i], wi = sw[i];
                    double2 *a = A22 + (size_t)i * F + j;
                    const double2 x = *a;
                    // v_i conj(w_j) + w_i conj(v_j)
                    const double re = vi.x * wj.x + vi.y * wj.y + wi.x * vj.x + wi.y * vj.y;
                    const double im = vi.y * wj.x - vi.x * wj.y + wi.y * vj.x - wi.x * vj.y;
                    *a = make_double2(x.x - re, x.y - im);
                }
            }
        } else {
            for (int i = 0; i < m; ++i)
                for (int j = t; j < m; j += kEigThreads) {
                    const double2 vi = sv[i], wi = sw[i], vj = sv[j], wj = sw[j];
                    double2 *a = A22 + (size_t)i * F + j;
                    const double2 x = *a;
                    const double re = vi.x * wj.x + vi.y * wj.y + wi.x * vj.x + wi.y * vj.y;
                    const double im = vi.y * wj.x - vi.x * wj.y + wi.y * vj.x - wi.x * vj.y;
                    *a = make_double2(x.x - re, x.y - im);
                }
        }
        __syncthreads();
    }
    if (t == 0) {
        d[F - 1] = A[(size_t)(F - 1) * F + (F - 1)].x;
        e[F - 1] = 0.0;
        if (F >= 1) tau[F - 1] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    // 2. All eigenvalues by bisection on Sturm counts (descending order).
    double lo_b = 1e300, hi_b = -1e300, emax = 0.0;
    for (int i = t; i < F; i += kEigThreads) {
        const double di = d[i];
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < F ? fabs(e[i]) : 0.0);
        lo_b = fmin(lo_b, di - r);
        hi_b = fmax(hi_b, di + r);
        sd[i] = di;
        se2[i] = (i + 1 < F) ? e[i] * e[i] : 0.0;
        emax = fmax(emax, se2[i]);
    }
    hi_b = block_max(hi_b, red);
    lo_b = -block_max(-lo_b, red);
    emax = block_max(emax, red);
    const double tnorm = fmax(fabs(lo_b), fabs(hi_b));
    const double pivmin = fmax(DBL_MIN, DBL_MIN * emax);
    lo_b -= 2.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
    hi_b += 2.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
    for (int idx = t; idx < F; idx += kEigThreads) {
        const int target = F - 1 - idx;
        double lo = lo_b, hi = hi_b;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (sturm_count(sd, se2, F, mid, pivmin) > target) hi = mid; else lo = mid;
        }
        lam[idx] = 0.5 * (lo + hi);
        if (evals_out) evals_out[(size_t)plane * F + idx] = lam[idx];
    }
    __syncthreads();
    if (c <= 0) return;

    // 3. Inverse iteration on T - lambda I for the c largest eigenvalues.
    //    Partial-pivoting LU of the tridiagonal; one thread per eigenvector.
    // scratch per vector: u0, u1, u2 (the three diagonals of U), ml (multipliers),
    // b (right-hand side, then the solution), sw (1 where rows were swapped)
    double *ts = tscratch + (size_t)plane * c * 6 * F;
    if (t < c) {
        double *u0 = ts + (size_t)t * 6 * F;
        double *u1 = u0 + F, *u2 = u1 + F, *ml = u2 + F, *b = ml + F, *sw_ = b + F;
        const double lm = lam[t];
        const double tiny = DBL_EPSILON * tnorm + pivmin;
        for (int i = 0; i < F; ++i) {
            u0[i] = sd[i] - lm;
            u1[i] = (i + 1 < F) ? e[i] : 0.0;
            u2[i] = 0.0;
            sw_[i] = 0.0;
        }
        for (int i = 0; i + 1 < F; ++i) {
            const double sub = e[i];
            if (fabs(u0[i]) >= fabs(sub)) {
                if (u0[i] == 0.0) u0[i] = tiny;
                ml[i] = sub / u0[i];
                u0[i + 1] -= ml[i] * u1[i];
            } else {
                // swap rows i and i+1, then eliminate
                const double l = u0[i] / sub;
                const double t1 = u0[i + 1];
                const double t2 = (i + 2 < F) ? u1[i + 1] : 0.0;
                u0[i] = sub;
                u0[i + 1] = u1[i] - l * t1;
                if (i + 2 < F) u1[i + 1] = -l * t2;
                u1[i] = t1;
                u2[i] = t2;
                ml[i] = l;
                sw_[i] = 1.0;
            }
        }
        if (u0[F - 1] == 0.0) u0[F - 1] = tiny;
        // deterministic start vector
        for (int i = 0; i < F; ++i) b[i] = 1.0 + 0.37 * sin(0.731 * i + 1.3 * t);
        for (int it = 0; it < 3; ++it) {
            for (int i = 0; i + 1 < F; ++i) {
                if (sw_[i] != 0.0) { const double tmp = b[i]; b[i] = b[i + 1]; b[i + 1] = tmp; }
                b[i + 1] -= ml[i] * b[i];
            }
            b[F - 1] /= u0[F - 1];
            if (F >= 2) b[F - 2] = (b[F - 2] - u1[F - 2] * b[F - 1]) / u0[F - 2];
            for (int i = F - 3; i >= 0; --i) b[i] = (b[i] - u1[i] * b[i + 1] - u2[i] * b[i + 2]) / u0[i];
            double nrm2 = 0.0;
            for (int i = 0; i < F; ++i) nrm2 += b[i] * b[i];
            const double inv = 1.0 / sqrt(nrm2);
            for (int i = 0; i < F; ++i) b[i] *= inv;
        }
    }
    __syncthreads();

    // 4. Orthonormalise the c tridiagonal eigenvectors (classical Gram-Schmidt,
    //    two passes), one vector at a time against the earlier ones.
    for (int i = 0; i < c; ++i) {
        double *bi = ts + (size_t)i * 6 * F + 4 * F;
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = 0; j < i; ++j) {
                const double *bj = ts + (size_t)j * 6 * F + 4 * F;
                double dot = 0.0;
                for (int q = t; q < F; q += kEigThreads) dot += bj[q] * bi[q];
                dot = block_sum(dot, red);
                for (int q = t; q < F; q += kEigThreads) bi[q] -= dot * bj[q];
                __syncthreads();
            }
        }
        double nrm2 = 0.0;
        for (int q = t; q < F; q += kEigThreads) nrm2 += bi[q] * bi[q];
        nrm2 = block_sum(nrm2, red);
        const double inv = 1.0 / sqrt(nrm2);
        for (int q = t; q < F; q += kEigThreads) bi[q] *= inv;
        __syncthreads();
    }

    // 5. Back-transform x = H_0 H_1 ... H_{F-2} y; one wave per vector.
    double2 *xs = xscratch + (size_t)plane * c * F;
    for (int i = t; i < c * F; i += kEigThreads) {
        const int vi = i / F, q = i % F;
        xs[i] = make_double2(ts[(size_t)vi * 6 * F + 4 * F + q], 0.0);
    }
    __syncthreads();
    const int lane = t & 63, wave = t >> 6;
    for (int vi = wave; vi < c; vi += kEigWaves) {
        double2 *x = xs + (size_t)vi * F;
        for (int k = F - 2; k >= 0; --k) {
            const double2 tk = tau[k];
            if (tk.x == 0.0 && tk.y == 0.0) continue;
            const int m = F - k - 1;
            const double2 *v = A + (size_t)k * F + k + 1;
            double sr = 0.0, si = 0.0;
            for (int q = lane; q < m; q += 64) {
                const double2 p = cconjmul(v[q], x[k + 1 + q]);
                sr += p.x;
                si += p.y;
            }
            sr = wave_sum(sr);
            si = wave_sum(si);
            const double2 s = cmul(tk, make_double2(sr, si));
            for (int q = lane; q < m; q += 64) {
                const double2 p = cmul(v[q], s);
                x[k + 1 + q] = make_double2(x[k + 1 + q].x - p.x, x[k + 1 + q].y - p.y);
            }
        }
    }
    __syncthreads();
    for (int i = t; i < c * F; i += kEigThreads) {
        const int vi = i % c, f = i / c;
        V[(size_t)f * c + vi] = xs[(size_t)vi * F + f];
    }
}

__global__ void clear_status_kernel(int *status, int *bar, int *eflag, int planes) {
    if (threadIdx.x == 0) *status = 0;
    for (int i = threadIdx.x; i < planes * kBarStride; i += blockDim.x) bar[i] = 0;
    for (int i = threadIdx.x; i < planes; i += blockDim.x) eflag[i] = 0;
}

// ---------------------------------------------------------------- removal
// I_f = I - (I V_c) V_c^H on v_mfma_f64_16x16x4f64, both products transposed so
// that the pixel is the MFMA's N index (a tile is 16 consecutive pixels):
//   Y^T   = W1 X^T        row 2 i (re) and 2 i + 1 (im) of Y^T = (I V_c)[p][i];
//                         K-step 2 q + r = frames 4 q .. 4 q + 3, their re (r = 0)
//                         or im (r = 1) parts
//   X_f^T = X^T - W2 Y^T  output tile tau = frames 8 tau .. 8 tau + 7: result
//                         register r of lane l = frame 8 tau + 2 (l / 16) + r / 2,
//                         re (r even) or im (r odd); K = the rows of Y^T, 4 a step
// W1 and W2 are V_c's entries laid out as A operands (lane l: row l % 16, K index
// l / 16), built per plane by removal_f64_tables_kernel, zero past 2c rows or F
// frames.  FP32 inputs are exact in FP64, so only FP64 summation rounds.  The
// first product's accumulators are the second's B operands as they stand:
// register r of lane l in tile T holds row 16 T + 4 r + l / 16 of Y^T, which is
// what lane l supplies for K-step 4 T + r.

// One thread per (plane, table entry, lane).
__global__ void removal_f64_tables_kernel(const double2 *__restrict__ V, double *__restrict__ tab,
                                          int F, int c, Removal64Dims d, int planes)
{
    const size_t n1 = (size_t)d.MT * d.KS1 * 64, n2 = (size_t)d.FT * d.KS2 * 64;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)planes * (n1 + n2)) return;
    const int plane = (int)(idx / (n1 + n2));
    const size_t e = idx % (n1 + n2);
    const double2 *Vp = V + (size_t)plane * F * c;
    const int lane = (int)(e % 64), m = lane & 15, k = lane >> 4;
    double val = 0.0;
    if (e < n1) {
        // W1: tile T, step t; row 16 T + m of Y^T against (frame, part) of X^T
        const int t = (int)((e / 64) % d.KS1), T = (int)(e / 64 / d.KS1);
        const int row = 16 * T + m, i = row >> 1, yim = row & 1;
        const int g = 4 * (t >> 1) + k, xim = t & 1;
        if (i < c && g < F) {
            const double2 v = Vp[(size_t)g * c + i];
            // re y = xr vr - xi vi,  im y = xr vi + xi vr
            val = yim ? (xim ? v.x : v.y) : (xim ? -v.y : v.x);
        }
    } else {
        // W2: output tile tau, step s; output row m (frame, part) against row 4 s + k of Y^T
        const size_t e2 = e - n1;
        const int s = (int)((e2 / 64) % d.KS2), tau = (int)(e2 / 64 / d.KS2);
        const int r = m >> 2, j = m & 3;
        const int g = 8 * tau + 2 * j + (r >> 1), oim = r & 1;
        const int yrow = 4 * s + k, i = yrow >> 1, yim = yrow & 1;
        if (i < c && g < F) {
            const double2 v = Vp[(size_t)g * c + i];
            // y conj(v): re = yr vr + yi vi,  im = yi vr - yr vi
            val = oim ? (yim ? v.x : -v.y) : (yim ? v.y : v.x);
        }
    }
    tab[(size_t)plane * (n1 + n2) + e] = val;
}

// A wave owns kRemNT tiles of 16 pixels (the table operands are shared by them);
// MT = tiles of 16 rows of Y^T.
constexpr int kRemNT = 2;
constexpr int kRemAhead = 4;       // frame groups of the plane in flight
template <int MT>
__global__ __launch_bounds__(256) void removal_f64_kernel(float2 *__restrict__ P,
                                                          const double *__restrict__ tab, int F,
                                                          int npix, Removal64Dims d,
                                                          const int *__restrict__ eflag)
{
    const int plane = blockIdx.y;
    if (eflag[plane]) return;      // non-finite covariance: the plane stays unfiltered
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n16 = lane & 15, k4 = lane >> 4;
    const int p0 = (blockIdx.x * 4 + wave) * 16 * kRemNT;
    if (p0 >= npix) return;
    float2 *X = P + (size_t)plane * F * npix;
    const double *W1 = tab + (size_t)plane * (d.t1_plane + d.t2_plane);
    const double *W2 = W1 + d.t1_plane;
    int px[kRemNT];
    bool pok[kRemNT];
#pragma unroll
    for (int nt = 0; nt < kRemNT; ++nt) {
        px[nt] = p0 + 16 * nt + n16;
        pok[nt] = px[nt] < npix;
    }

    // Y^T = W1 X^T: four frames per pair of K-steps.  The plane is read from
    // HBM kRemAhead frame groups ahead (a ring of registers, the loop unrolled
    // by its depth); the table operands (L2) one group ahead.
    f64x4 y[MT][kRemNT];
#pragma unroll
    for (int T = 0; T < MT; ++T)
#pragma unroll
        for (int nt = 0; nt < kRemNT; ++nt) y[T][nt] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int nq = d.KS1 / 2;
    // past the last group the frame index is >= F: zeros, nothing read
    auto load_x = [&](int q, float2 (&x)[kRemNT]) {
        const int g = 4 * q + k4;
#pragma unroll
        for (int nt = 0; nt < kRemNT; ++nt)
            x[nt] = (g < F && pok[nt]) ? X[(size_t)g * npix + px[nt]] : make_float2(0.f, 0.f);
    };
    auto load_w1 = [&](int q, double (&a)[MT][2]) {
        const int qq = min(q, nq - 1);
#pragma unroll
        for (int T = 0; T < MT; ++T) {
            a[T][0] = W1[((size_t)T * d.KS1 + 2 * qq) * 64 + lane];
            a[T][1] = W1[((size_t)T * d.KS1 + 2 * qq + 1) * 64 + lane];
        }
    };
    float2 xr[kRemAhead][kRemNT];
    double aw[2][MT][2];
#pragma unroll
    for (int u = 0; u < kRemAhead; ++u) load_x(u, xr[u]);
    load_w1(0, aw[0]);
    for (int q0 = 0; q0 < nq; q0 += kRemAhead) {
#pragma unroll
        for (int u = 0; u < kRemAhead; ++u) {
            const int q = q0 + u;
            if (q < nq) {
                load_w1(q + 1, aw[(u + 1) & 1]);
#pragma unroll
                for (int T = 0; T < MT; ++T)
#pragma unroll
                    for (int nt = 0; nt < kRemNT; ++nt) {
                        y[T][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[u & 1][T][0], (double)xr[u][nt].x, y[T][nt], 0, 0, 0);
                        y[T][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[u & 1][T][1], (double)xr[u][nt].y, y[T][nt], 0, 0, 0);
                    }
                load_x(q + kRemAhead, xr[u]);
            }
        }
    }

    // X_f^T = X^T - W2 Y^T, 8 frames per output tile; the inputs of the tile
    // two ahead (read from HBM) are requested before this tile's products
    auto load_out = [&](int tau, float2 (&x)[2][kRemNT]) {
        const int g0 = 8 * tau + 2 * k4;
#pragma unroll
        for (int nt = 0; nt < kRemNT; ++nt) {
            x[0][nt] = (g0 < F && pok[nt]) ? X[(size_t)g0 * npix + px[nt]] : make_float2(0.f, 0.f);
            x[1][nt] = (g0 + 1 < F && pok[nt]) ? X[(size_t)(g0 + 1) * npix + px[nt]] : make_float2(0.f, 0.f);
        }
    };
    float2 xo[2][2][kRemNT];
    load_out(0, xo[0]);
    load_out(1, xo[1]);
    for (int t0 = 0; t0 < d.FT; t0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int tau = t0 + u;
            if (tau < d.FT) {
                f64x4 o[kRemNT];
#pragma unroll
                for (int nt = 0; nt < kRemNT; ++nt) o[nt] = f64x4{0.0, 0.0, 0.0, 0.0};
                const double *w2 = W2 + (size_t)tau * d.KS2 * 64 + lane;
#pragma unroll
                for (int T = 0; T < MT; ++T)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double a = w2[(size_t)(4 * T + r) * 64];
#pragma unroll
                        for (int nt = 0; nt < kRemNT; ++nt)
                            o[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, y[T][nt][r], o[nt], 0, 0, 0);
                    }
                const int g0 = 8 * tau + 2 * k4;
#pragma unroll
                for (int nt = 0; nt < kRemNT; ++nt) {
                    if (!pok[nt]) continue;
                    const float2 x0 = xo[u][0][nt], x1 = xo[u][1][nt];
                    if (g0 < F)
                        X[(size_t)g0 * npix + px[nt]] = make_float2((float)((double)x0.x - o[nt][0]),
                                                                    (float)((double)x0.y - o[nt][1]));
                    if (g0 + 1 < F)
                        X[(size_t)(g0 + 1) * npix + px[nt]] = make_float2((float)((double)x1.x - o[nt][2]),
                                                                          (float)((double)x1.y - o[nt][3]));
                }
                load_out(tau + 2, xo[u]);
            }
        }
    }
}

// ---------------------------------------------------------------- removal, BF16 split
// Split-precision form of I_f = I - (I V_c) V_c^H on v_mfma_f32_32x32x16_bf16.
// A wave owns 32 pixels and forms both products transposed, so that the pixel
// is the MFMA's N index (lanes read and write consecutive pixels):
//   Y^T   = W1 X^T         rows 2i, 2i+1 = (re, im) of (I V_c)[p][i];
//                          K = (frame, re/im), 8 frames per K-step
//   X_f^T = X^T - W2 Y^T   rows = frames (one real, one imaginary accumulator);
//                          K = the 2c real rows of Y^T
// W1 and W2 hold the clutter eigenvectors arranged as MFMA A operands, built
// per plane by removal_tables_kernel.  Every operand is a sum of kSplitTerms = 3
// BF16 terms (hi + mid + lo, exact for FP32 data); the products of terms whose
// orders add up to less than three are accumulated in FP32, and the first
// product's accumulators are added into FP64 after every K-step.  The first
// product's output feeds the second product's B operand from registers: a
// lane's accumulator q holds row 8 (q / 4) + 4 half + q % 4 of its 32-row
// tile, so K-step t of the second product (tile t / 2, half t % 2) takes
// accumulators 8 (t % 2) .. 8 (t % 2) + 7, and W2 orders its K index alike.



// One thread per (plane, table entry, lane): the 8 BF16 values of the lane's
// operand, in kSplitTerms terms.
__global__ void removal_tables_kernel(const double2 *__restrict__ V, bf16x8 *__restrict__ tab,
                                      int F, int c, RemovalDims d, int planes)
{
    constexpr int NT = kSplitTerms;
    const size_t n1 = (size_t)d.MT * d.S1 * 64, n2 = (size_t)d.FT * d.KT2 * 2 * 64;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)planes * (n1 + n2)) return;
    const int plane = (int)(idx / (n1 + n2));
    const size_t e = idx % (n1 + n2);
    const double2 *Vp = V + (size_t)plane * F * c;
    bf16x8 *out = tab + (size_t)plane * (d.t1_plane + d.t2_plane);
    const int lane = (int)(e % 64), h = lane >> 5, row = lane & 31;
    double val[8];
    size_t base;
    if (e < n1) {
        // W1: row m = (i, part), K index j = (frame 8 s + 4 h + j / 2, re/im j % 2)
        const int s = (int)((e / 64) % d.S1), mt = (int)(e / (64 * (size_t)d.S1));
        const int m = 32 * mt + row, i = m >> 1, part = m & 1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int g = 8 * s + 4 * h + (j >> 1), ri = j & 1;
            double x = 0.0;
            if (i < c && g < F) {
                const double2 v = Vp[(size_t)g * c + i];
                // Y_re = sum x_re v_re - x_im v_im,  Y_im = sum x_re v_im + x_im v_re
                x = part == 0 ? (ri == 0 ? v.x : -v.y) : (ri == 0 ? v.y : v.x);
            }
            val[j] = x;
        }
        base = ((size_t)mt * d.S1 + s) * NT * 64 + lane;
    } else {
        // W2: row = frame f, K index j = row r of Y^T (see above); ro = 0 real
        // output, 1 imaginary output
        const size_t e2 = e - n1;
        const int ro = (int)((e2 / 64) % 2), t = (int)((e2 / 128) % d.KT2);
        const int ft = (int)(e2 / (128 * (size_t)d.KT2));
        const int f = 32 * ft + row, mt = t >> 1, tl = t & 1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = 32 * mt + 8 * (2 * tl + (j >> 2)) + 4 * h + (j & 3);
            const int i = r >> 1, part = r & 1;
            double x = 0.0;
            if (i < c && f < F) {
                const double2 v = Vp[(size_t)f * c + i];
                // (Y conj(v))_re = Y_re v_re + Y_im v_im,  _im = Y_im v_re - Y_re v_im
                x = ro == 0 ? (part == 0 ? v.x : v.y) : (part == 0 ? -v.y : v.x);
            }
            val[j] = x;
        }
        base = d.t1_plane + (((size_t)ft * d.KT2 + t) * 2 + ro) * NT * 64 + lane;
    }
    bf16x8 o[NT];
#pragma unroll
    for (int j = 0; j < 8; ++j) ULM_SET3(o, j, val[j]);
#pragma unroll
    for (int k = 0; k < NT; ++k) out[base + (size_t)k * 64] = o[k];
}

template <int MT>
__global__ __launch_bounds__(256) void removal_bf16_kernel(float2 *__restrict__ P,
                                                           const bf16x8 *__restrict__ tab, int F,
                                                           int npix, RemovalDims d,
                                                           const int *__restrict__ eflag)
{
    constexpr int NT = kSplitTerms;
    const int plane = blockIdx.y;
    if (eflag[plane]) return;      // non-finite covariance: the plane stays unfiltered
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, n = lane & 31;
    const int p0 = (blockIdx.x * 4 + wave) * 32;
    if (p0 >= npix) return;
    const int p = p0 + n;
    const bool pin = p < npix;
    const int pc = pin ? p : npix - 1;
    float2 *X = P + (size_t)plane * F * npix;
    const bf16x8 *t1 = tab + (size_t)plane * (d.t1_plane + d.t2_plane) + lane;
    const bf16x8 *t2 = t1 + d.t1_plane;

    // first product, Y^T = W1 X^T: this lane's B operand at K-step s is
    // frames 8 s + 4 h + [0, 4) of pixel p, (re, im) each
    double y[MT][16];
    f32x16 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int q = 0; q < 16; ++q) y[mt][q] = 0.0;
        acc[mt] = f32x16{};
    }
    float2 cur[4], nxt[4];
    auto fetch = [&](int s, float2 *dst) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int g = 8 * s + 4 * h + q;
            const float2 v = X[(size_t)min(g, F - 1) * npix + pc];
            dst[q] = (g < F && pin) ? v : make_float2(0.f, 0.f);
        }
    };
    fetch(0, cur);
    for (int s = 0; s < d.S1; ++s) {
        if (s + 1 < d.S1) fetch(s + 1, nxt);
        bf16x8 b[NT];
        {
            bf16x2x3 t[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] = split3x2(f32x2{cur[q].x, cur[q].y});
            b[0] = cat4(t[0].h, t[1].h, t[2].h, t[3].h);
            b[1] = cat4(t[0].m, t[1].m, t[2].m, t[3].m);
            b[2] = cat4(t[0].l, t[1].l, t[2].l, t[3].l);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const bf16x8 *w = t1 + ((size_t)mt * d.S1 + s) * NT * 64;
            bf16x8 a[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) a[k] = w[k * 64];
#pragma unroll
            for (int ord = NT - 1; ord >= 0; --ord)          // smallest products first
#pragma unroll
                for (int ta = 0; ta <= ord; ++ta)
                    acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ta], b[ord - ta], acc[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int q = 0; q < 16; ++q) y[mt][q] += (double)acc[mt][q];
            acc[mt] = f32x16{};
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
    }

    // second product, one 32-frame tile at a time: B operand of K-step t =
    // accumulator rows 8 (t % 2) .. + 7 of tile t / 2, split into terms
    bf16x8 b2[2 * MT][NT];
#pragma unroll
    for (int t = 0; t < 2 * MT; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            ULM_SET3(b2[t], j, y[t >> 1][8 * (t & 1) + j]);
    for (int ft = 0; ft < d.FT; ++ft) {
        float2 x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int f = 32 * ft + 8 * (q >> 2) + 4 * h + (q & 3);
            x[q] = X[(size_t)min(f, F - 1) * npix + pc];
        }
        f32x16 are = {}, aim = {};
#pragma unroll
        for (int t = 0; t < 2 * MT; ++t) {
            if (t >= d.KT2) break;
            const bf16x8 *w = t2 + (((size_t)ft * d.KT2 + t) * 2) * NT * 64;
            bf16x8 ar[NT], ai[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                ar[k] = w[k * 64];
                ai[k] = w[(NT + k) * 64];
            }
#pragma unroll
            for (int ord = NT - 1; ord >= 0; --ord)          // smallest products first
#pragma unroll
                for (int ta = 0; ta <= ord; ++ta) {
                    are = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ta], b2[t][ord - ta], are, 0, 0, 0);
                    aim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[ta], b2[t][ord - ta], aim, 0, 0, 0);
                }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int f = 32 * ft + 8 * (q >> 2) + 4 * h + (q & 3);
            if (f < F && pin) X[(size_t)f * npix + p] = make_float2(x[q].x - are[q], x[q].y - aim[q]);
        }
    }
}

hipError_t launch_filter(const ulm_ctx *ctx, float2 *proj, double *eigvals_out, char *ws,
                         hipStream_t st)
{
    const Geometry &g = ctx->geo;
    const Workspace &w = ctx->ws;
    const int F = g.n_frames, npix = g.nz * g.nu, planes = g.n_planes;
    const int c = ctx->cfg.svd_cutoff;
    const int nblk = cdiv(F, kGramBlock);
    double2 *part = (double2 *)(ws + w.gram_part);
    double2 *C = (double2 *)(ws + w.cov);
    int *status = (int *)(ws + w.status);

    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, st, status, (int *)(ws + w.bar),
                       (int *)(ws + w.eflag), planes);
    const int nwg = planes * w.gram_pairs * w.gram_chunks;
    if (ctx->cfg.precision == ULM_PREC_BF16X3)
        hipLaunchKernelGGL(gram_bf16x3_kernel, dim3(nwg), dim3(256), 0, st, proj, part, F, npix,
                           w.gram_pairs, w.gram_chunks, nblk);
    else
        hipLaunchKernelGGL(gram_f64_kernel, dim3(nwg), dim3(256), 0, st, proj, part, F, npix,
                           w.gram_pairs, w.gram_chunks, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(planes * w.gram_pairs * (kGramBlock / kReduceRows)),
                       dim3(256), 0, st, part, C, F, w.gram_pairs, w.gram_chunks, nblk);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    double *evals = (double *)(ws + w.evals);
    if (eigen_coop_lds(F, c) <= 150 * 1024) {
        EigArgs a;
        a.C = C;
        a.H = (double2 *)(ws + w.hvec);
        a.tau = (double2 *)(ws + w.tau);
        a.d = (double *)(ws + w.diag);
        a.e = (double *)(ws + w.offd);
        a.lam = evals;
        a.lam_out = eigvals_out;
        a.V = (double2 *)(ws + w.evecs);
        a.tscr = (double *)(ws + w.tscratch);
        a.xscr = (double2 *)(ws + w.xscratch);
        a.vbuf = (double2 *)(ws + w.vbuf);
        a.pbuf = (double2 *)(ws + w.pbuf);
        a.bar = (int *)(ws + w.bar);
        a.flag = (int *)(ws + w.eflag);
        a.status = status;
        a.F = F;
        a.c = c;
        a.W = eigen_coop_width(F);
        // diagnostic switch: the fenced exchange mode even where a plane's
        // work-groups share one XCD (the results are the same bit for bit)
        a.agent_scope = getenv("ULMPROJ_EIGEN_AGENT_SCOPE") != nullptr;
        a.planes = planes;
        a.plane0 = 0;
        if ((e = launch_eigen_coop(a, st)) != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(eigen_kernel, dim3(planes), dim3(kEigThreads), 0, st, C,
                           (double2 *)(ws + w.tau), (double *)(ws + w.diag), (double *)(ws + w.offd),
                           evals, (double2 *)(ws + w.evecs), (double *)(ws + w.tscratch),
                           (double2 *)(ws + w.xscratch), F, c, status, eigvals_out, (int *)(ws + w.eflag));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (c > 0 && ctx->cfg.precision == ULM_PREC_BF16X3) {
        const RemovalDims rd = removal_dims(F, c);
        bf16x8 *tab = (bf16x8 *)(ws + w.rtab);
        const size_t nthr = (size_t)planes * (rd.t1_plane + rd.t2_plane) / kSplitTerms;
        hipLaunchKernelGGL(removal_tables_kernel, dim3((unsigned)cdiv<size_t>(nthr, 256)), dim3(256), 0,
                           st, (const double2 *)(ws + w.evecs), tab, F, c, rd, planes);
        dim3 grid(cdiv(npix, 128), planes);
        const int *eflag = (const int *)(ws + w.eflag);
        if (rd.MT == 1)
            hipLaunchKernelGGL(removal_bf16_kernel<1>, grid, dim3(256), 0, st, proj, tab, F, npix, rd, eflag);
        else
            hipLaunchKernelGGL(removal_bf16_kernel<2>, grid, dim3(256), 0, st, proj, tab, F, npix, rd, eflag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (c > 0) {
        const Removal64Dims rd = removal64_dims(F, c);
        double *tab = (double *)(ws + w.rtab64);
        const size_t nthr = (size_t)planes * (rd.t1_plane + rd.t2_plane);
        hipLaunchKernelGGL(removal_f64_tables_kernel, dim3((unsigned)cdiv<size_t>(nthr, 256)), dim3(256), 0,
                           st, (const double2 *)(ws + w.evecs), tab, F, c, rd, planes);
        dim3 grid(cdiv(npix, 4 * 16 * kRemNT), planes);
        const int *eflag = (const int *)(ws + w.eflag);
        switch (rd.MT) {
            case 1: hipLaunchKernelGGL(removal_f64_kernel<1>, grid, dim3(256), 0, st, proj, tab, F, npix, rd, eflag); break;
            case 2: hipLaunchKernelGGL(removal_f64_kernel<2>, grid, dim3(256), 0, st, proj, tab, F, npix, rd, eflag); break;
            case 3: hipLaunchKernelGGL(removal_f64_kernel<3>, grid, dim3(256), 0, st, proj, tab, F, npix, rd, eflag); break;
            default: hipLaunchKernelGGL(removal_f64_kernel<4>, grid, dim3(256), 0, st, proj, tab, F, npix, rd, eflag); break;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ulm
