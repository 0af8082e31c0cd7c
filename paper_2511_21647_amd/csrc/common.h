// Internal definitions shared by the HIP translation units of libulmproj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ulmproj.h"

namespace ulm {

constexpr int kDasThreads = 256;   // one pixel per thread
constexpr int kDasTileU = 32;      // tile: 8 rows (z) x 32 columns (u)
constexpr int kDasTileZ = 8;
constexpr int kDasFrames = 16;     // frames beamformed per delay evaluation

constexpr int kFirTileZ = 64;      // stage-2 tile: 64 rows (8 per thread) x 32 columns
constexpr int kFirTileU = 32;
static_assert(8 * (256 / kFirTileU) == kFirTileZ, "stage-2 tile: 8 rows per thread");
constexpr int kFirMaxTaps = 48;
constexpr int kFirGroup = 4;       // slabs per stage-2 work-group (many-slab projections)

constexpr int kGramBlock = 64;     // frames per Gram block (rows and columns)
constexpr int kGramChunk = 2048;   // pixels reduced by one Gram work-group
constexpr int kGramStage = 32;     // pixels staged in LDS per step

constexpr int kNccBand = 16;       // NCC output rows per work-group
constexpr int kNccMaxHalf = 7;     // template half-width limit (size <= 15)

// Split-precision clutter filter: BF16 terms per operand (x = hi + mid + lo),
// and the shape of the removal's per-plane MFMA operand tables (built from the
// clutter eigenvectors), counted in 16-byte lane operands (8 BF16 values).
constexpr int kSplitTerms = 3;
// FP64 removal on the matrix cores (16 x 16 x 4 tiles): operand tables per plane.
struct Removal64Dims {
    int MT;            // 16-row tiles of the 2c real rows of (I V_c)^T (c <= 32: at most 4)
    int KS1;           // K-steps of I V_c: (re, im) per 4 frames
    int FT;            // 8-frame tiles of the output
    int KS2;           // K-steps (4 real rows each, all MT tiles) of (I V_c) V_c^H
    size_t t1_plane;   // doubles per plane, first product
    size_t t2_plane;   // doubles per plane, second product
};
inline Removal64Dims removal64_dims(int F, int c) {
    Removal64Dims d;
    d.MT = (2 * c + 15) / 16;
    d.KS1 = 2 * ((F + 3) / 4);
    d.FT = (F + 7) / 8;
    d.KS2 = 4 * d.MT;
    d.t1_plane = (size_t)d.MT * d.KS1 * 64;
    d.t2_plane = (size_t)d.FT * d.KS2 * 64;
    return d;
}

struct RemovalDims {
    int MT;            // 32-row tiles of the 2c real rows of (I V_c)^T
    int S1;            // K-steps (8 frames each) of I V_c
    int FT;            // 32-frame tiles of the output
    int KT2;           // K-steps (16 real rows each) of (I V_c) V_c^H
    size_t t1_plane;   // lane operands per plane, first product
    size_t t2_plane;   // lane operands per plane, second product
};
inline RemovalDims removal_dims(int F, int c) {
    RemovalDims d;
    d.MT = (2 * c + 31) / 32;
    d.S1 = (F + 7) / 8;
    d.FT = (F + 31) / 32;
    d.KT2 = (2 * c + 15) / 16;
    d.t1_plane = (size_t)d.MT * d.S1 * kSplitTerms * 64;
    d.t2_plane = (size_t)d.FT * d.KT2 * 2 * kSplitTerms * 64;
    return d;
}

// Status bits written to the workspace status word.
constexpr int kStatusNumeric = 1;   // a plane's covariance was not finite: plane left unfiltered
constexpr int kStatusBarrier = 2;   // the eigensolver's inter-work-group wait timed out
constexpr int kStatusCnnRow = 4;    // a CNN decode row held more peaks than its staging slot

struct Geometry {
    int n_elem, n_samp, n_frames, n_angles;
    int nu, nz, n_blocks, n_planes;
    float pitch, fs_over_c, f0_over_c, t_start_fs;
    float du, dz, u0, z0;
};

// Device tables owned by the context.
struct Tables {
    float *stx;        // [K][Nz]   fractional part of (tau_tx(v_ref, z; k) + z / c - t_start) * fs
    int *sti;          // [K][Nz]   its integer part
    float2 *phz;       // [K][Nz]   exp(i 2 pi f0 (tau_tx - z / c))
    float *rxd;        // [Nc][Nz*Nu] (r - z) * fs / c
    float2 *rxp;       // [Nc][Nz*Nu] exp(i 2 pi f0 (r - z) / c)
    int *win;          // [K][tiles][Nc] DAS window: first staged sample * 16 + (16-sample chunks - 1)
    int das_len;       // staged samples per window (64 or 128)
    float2 *taps;      // [K][B][T] stage-2 axial FIR taps (first meta.y used)
    int2 *tap_meta;    // [K][B]    (first tap offset, number of taps)
    double *angles;    // [K]       steering angles (simulator)
    int n_taps;        // maximum taps over (transmit, block)
    int fir_group;     // slabs per stage-2 work-group: 1 or kFirGroup
    float2 *sep_tw;    // MB-separation FFT twiddles for F frames (null if F has a factor > 7)
    int *xd_n;         // [K][Nu] cross projection: integer part of the axial shift of column i
    float4 *xd_w;      // [K][Nu] ((1 - frac) e, frac e), e = the column's stage-2 phase
                       // (both null unless the v grid equals the u grid)
    int xd_nmin, xd_nmax;   // range of xd_n
};

// Words per plane of the eigensolver's barrier area: one grid-barrier flag per
// work-group (at most 32), and in the last word the set of XCDs (XCC ids) the
// plane's work-groups run on.
constexpr int kBarStride = 64;

// Offsets of the workspace regions, in bytes.
struct Workspace {
    size_t slices;      // [2][K][F][Nz][Nu] c64    stage-1 reference slices
    size_t gram_part;   // [planes][pairs][chunks][64][64] c128
    size_t cov;         // [planes][F][F] c128
    size_t tau;         // [planes][F] c128         Householder scalars
    size_t diag;        // [planes][F] f64
    size_t offd;        // [planes][F] f64
    size_t evals;       // [planes][F] f64          descending
    size_t evecs;       // [planes][F][c] c128
    size_t rtab64;      // [planes][t1_plane + t2_plane] f64 operands (FP64 removal)
    size_t rtab;        // [planes][t1_plane + t2_plane] BF16 x 8 operands (split removal only)
    size_t xprof;       // [2][K][B][F][Nz] c64 slab sums of the stage-1 slices (cross projection)
    size_t tscratch;    // [planes][c][6][F] f64    inverse-iteration scratch
    size_t xscratch;    // [planes][c][F] c128      back-transformed vectors
    size_t hvec;        // [planes][F][F] c128      Householder vectors
    size_t vbuf, pbuf;  // [planes][2][F] c128      column / p exchange (by step parity)
    size_t bar;         // [planes][kBarStride] i32 grid-barrier flags + XCC mask
    size_t eflag;       // [planes] i32
    size_t fmax;        // [planes][F] f32
    size_t band_cnt;    // [planes][F][bands] i32
    size_t band_off;    // [planes][F][bands] i32
    size_t staged;      // [planes][F][bands][cap] ulm_loc_t
    size_t status;      // i32
    size_t total;
    int gram_pairs, gram_chunks, bands, band_cap;
};

template <typename T> __host__ __device__ inline T cdiv(T a, T b) { return (a + b - 1) / b; }

// Columns of the padded clutter subspace the removal kernel is compiled for.

// Work-group remap so that consecutive logical work-groups land on the same
// XCD (the dispatcher deals work-groups round-robin over the 8 XCDs), so
// work-groups that read the same data share one L2.
__device__ inline int xcd_remap(int lin, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = lin & 7, s = lin >> 3;
    return x * q + min(x, r) + s;
}

}  // namespace ulm

struct ulm_ctx {
    ulm_config_t cfg;
    ulm::Geometry geo;
    ulm::Tables tab;
    ulm::Workspace ws;
    int device;
    hipEvent_t ev[4];
};
