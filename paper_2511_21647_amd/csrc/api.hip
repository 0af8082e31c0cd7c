// C ABI of libulmproj: configuration checks, per-geometry tables (computed on
// the host in FP64), workspace layout and the entry points.
#include "common.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <new>
#include <string>
#include <vector>

namespace ulm {
hipError_t launch_stage1(const ulm_ctx *ctx, const float2 *iq, float2 *slices, hipStream_t st);
hipError_t launch_stage2(const ulm_ctx *ctx, const float2 *slices, float2 *proj, hipStream_t st);
hipError_t launch_filter(const ulm_ctx *ctx, float2 *proj, double *eigvals_out, char *ws,
                         hipStream_t st);
hipError_t launch_localize(const ulm_ctx *ctx, const float2 *filt, ulm_loc_t *locs, int capacity,
                           int *count, char *ws, hipStream_t st);
hipError_t launch_density(const ulm_ctx *ctx, const ulm_loc_t *locs, const int *count,
                          int capacity, int up, uint32_t *dens, hipStream_t st);
hipError_t launch_sim(const ulm_ctx *ctx, const double *pos, const double *amp, int n_scat,
                      uint64_t seed, double noise_sigma, float *iq, const double *angles_dev,
                      hipStream_t st);
size_t ncc_lds_bytes(int nu, int half);
hipError_t launch_frame_max(const float2 *P, float *fmax, int n_img, int npix, hipStream_t st);
size_t cnn_workspace_bytes(int B, int H, int W, bool fp32, bool train);
size_t pair_workspace_bytes(int planes, int F, int capacity);
hipError_t launch_pairing(const ulm_ctx *ctx, const ulm_loc_t *locs, const int *count,
                          int capacity, ulm_loc3d_t *out, int out_capacity, int *out_count,
                          char *pws, hipStream_t st);
size_t motion_workspace_bytes(const Geometry &g, int L);
size_t motion_lds_bytes(const Geometry &g, int L);
hipError_t launch_motion(const ulm_ctx *ctx, const float2 *S, int ref, int L, float *disp,
                         float *motion, char *mws, hipStream_t st);
bool separate_supported(int F);
std::vector<float2> separate_twiddles(int F);
hipError_t launch_separate(const ulm_ctx *ctx, const float2 *P, int n_speed, float2 *out,
                           hipStream_t st);
size_t cnn_loc_workspace_bytes(int batch, int H, int W, int n_img, bool fp32);
hipError_t scratch_init(int device);
bool cross_supported(const Geometry &g, int per);
hipError_t launch_cross(const ulm_ctx *ctx, const float2 *slices, float2 *prof, float2 *Q,
                        hipStream_t st);
hipError_t launch_xdoppler(const ulm_ctx *ctx, const float2 *P, const float2 *Q, int window,
                           float2 *out, hipStream_t st);
void *scratch_ptr(int device);
hipError_t cnn_images(const float2 *P, const float *fmax, float *x0, int npix, int n0, int nb,
                      hipStream_t st);
hipError_t cnn_forward_heat(const float *params, const float *x0, float *heat, int B, int H, int W,
                            bool fp32, char *ws, hipStream_t st);
hipError_t cnn_gradients(const float *params, const float *x0, const float *mb_zu,
                         const int *mb_img, int n_mb, int B, int H, int W, bool fp32, float *grad,
                         float *loss, char *ws, hipStream_t st);
float *cnn_ws_grad(int B, int H, int W, bool fp32, char *ws);
hipError_t cnn_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                    hipStream_t st);
hipError_t cnn_localize(const float *params, const float2 *P, const float *fmax, float thr,
                        int n_img, int F, int H, int W, int batch, bool fp32, ulm_loc_t *locs,
                        int capacity, int *count, int *status, char *cws, hipStream_t st);
}  // namespace ulm

using namespace ulm;

static thread_local std::string g_err;

static int32_t fail(int32_t code, const std::string &msg) {
    g_err = msg;
    return code;
}

static int32_t hip_fail(hipError_t e, const char *where) {
    return fail(ULM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                     \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

extern "C" const char *ulm_last_error(void) { return g_err.c_str(); }

static void free_tables(ulm_ctx *ctx) {
    Tables &t = ctx->tab;
    void *ptrs[] = {t.stx, t.sti, t.phz, t.rxd, t.rxp, t.win, t.taps, t.tap_meta, t.angles, t.sep_tw,
                    t.xd_n, t.xd_w};
    for (void *p : ptrs) (void)hipFree(p);
}

static int32_t validate(const ulm_config_t &c) {
    // stage 1 reads runs of five samples of a record
    if (c.n_elem < 1 || c.n_samp < 5 || c.n_frames < 1) return fail(ULM_ERR_INVALID_ARG, "n_elem, n_samp (at least 5), n_frames");
    if (c.n_angles < 1 || c.n_angles > ULM_MAX_ANGLES) return fail(ULM_ERR_INVALID_ARG, "n_angles out of [1, 32]");
    if (c.n_frames > 1024) return fail(ULM_ERR_INVALID_ARG, "n_frames > 1024");
    if (c.nu < 1 || c.nz < 1 || c.nv < 1 || c.n_blocks < 1 || c.n_blocks > c.nv)
        return fail(ULM_ERR_INVALID_ARG, "grid sizes");
    if (!(c.pitch > 0 && c.c > 0 && c.f0 > 0 && c.fs > 0 && c.du > 0 && c.dz > 0 && c.dv > 0))
        return fail(ULM_ERR_INVALID_ARG, "non-positive physical constant");
    if (c.svd_cutoff < 0 || c.svd_cutoff > 32 || c.svd_cutoff > c.n_frames)
        return fail(ULM_ERR_INVALID_ARG, "svd_cutoff out of [0, min(32, n_frames)]");
    if (c.ncc_size < 3 || c.ncc_size > 2 * kNccMaxHalf + 1 || (c.ncc_size & 1) == 0)
        return fail(ULM_ERR_INVALID_ARG, "ncc_size must be odd in [3, 15]");
    if (!(c.sigma_u > 0 && c.sigma_z > 0)) return fail(ULM_ERR_INVALID_ARG, "template sigma");
    if (c.precision != ULM_PREC_FP64GRAM && c.precision != ULM_PREC_BF16X3)
        return fail(ULM_ERR_INVALID_ARG, "precision");
    for (int k = 0; k < c.n_angles; ++k)
        if (!(fabs(c.angles_rad[k]) < 1.2)) return fail(ULM_ERR_INVALID_ARG, "steering angle");
    if (c.z0 <= 0) return fail(ULM_ERR_INVALID_ARG, "z0 must be positive");
    if (ncc_lds_bytes(c.nu, (c.ncc_size - 1) / 2) > 160 * 1024)
        return fail(ULM_ERR_INVALID_ARG, "nu too large for the NCC band tile");
    if ((size_t)2 * 8 * c.n_samp * sizeof(float) > 160 * 1024)
        return fail(ULM_ERR_INVALID_ARG, "n_samp too large for the simulator");
    return ULM_OK;
}

// the cross projection (XDoppler) needs the v grid to equal the u grid: the
// plane's lateral axis is then the other orientation's v axis
static bool square_grid(const ulm_config_t &c) {
    return c.nv == c.nu && c.dv == c.du && c.v0 == c.u0;
}

static void layout_workspace(ulm_ctx *ctx) {
    const ulm_config_t &c = ctx->cfg;
    Workspace &w = ctx->ws;
    const size_t F = c.n_frames, planes = 2 * (size_t)c.n_blocks, npix = (size_t)c.nz * c.nu;
    const int nblk = cdiv(c.n_frames, kGramBlock);
    w.gram_pairs = nblk * (nblk + 1) / 2;
    w.gram_chunks = cdiv((int)npix, kGramChunk);
    w.bands = cdiv(c.nz, kNccBand);
    w.band_cap = cdiv(kNccBand, 2) * cdiv(c.nu, 2);
    const size_t cc = std::max(1, c.svd_cutoff);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    w.slices = take(sizeof(float2) * 2 * c.n_angles * F * npix);
    w.gram_part = take(sizeof(double2) * planes * w.gram_pairs * w.gram_chunks * kGramBlock * kGramBlock);
    w.cov = take(sizeof(double2) * planes * F * F);
    w.tau = take(sizeof(double2) * planes * F);
    w.diag = take(sizeof(double) * planes * F);
    w.offd = take(sizeof(double) * planes * F);
    w.evals = take(sizeof(double) * planes * F);
    w.evecs = take(sizeof(double2) * planes * F * cc);
    if (c.precision != ULM_PREC_BF16X3 && c.svd_cutoff > 0) {
        const Removal64Dims rd = removal64_dims(c.n_frames, c.svd_cutoff);
        w.rtab64 = take(sizeof(double) * planes * (rd.t1_plane + rd.t2_plane));
    } else {
        w.rtab64 = take(0);
    }
    if (c.precision == ULM_PREC_BF16X3 && c.svd_cutoff > 0) {
        const RemovalDims rd = removal_dims(c.n_frames, c.svd_cutoff);
        w.rtab = take(16 * planes * (rd.t1_plane + rd.t2_plane));
    } else {
        w.rtab = take(0);
    }
    w.xprof = take(square_grid(c) ? sizeof(float2) * 2 * c.n_angles * c.n_blocks * F * c.nz : 0);
    w.tscratch = take(sizeof(double) * planes * cc * 6 * F);
    w.xscratch = take(sizeof(double2) * planes * cc * F);
    w.hvec = take(sizeof(double2) * planes * F * F);
    w.vbuf = take(sizeof(double2) * planes * 2 * F);
    w.pbuf = take(sizeof(double2) * planes * 2 * F);
    w.bar = take(sizeof(int) * planes * kBarStride);
    w.eflag = take(sizeof(int) * planes);
    w.fmax = take(sizeof(float) * planes * F);
    w.band_cnt = take(sizeof(int) * planes * F * w.bands);
    w.band_off = take(sizeof(int) * planes * F * w.bands);
    w.staged = take(sizeof(ulm_loc_t) * planes * F * w.bands * w.band_cap);
    w.status = take(sizeof(int) * 4);
    w.total = off;
}

extern "C" int32_t ulm_create(const ulm_config_t *cfg, ulm_ctx_t **out) {
    if (!cfg || !out) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    int32_t rc = validate(*cfg);
    if (rc != ULM_OK) return rc;
    const ulm_config_t &c = *cfg;

    // stage-1 tables (FP64 on the host, rounded to FP32):
    //   (tau_tx(v_ref, z) + z / c - t_start) fs = sti[k][z] + stx[k][z]  (integer + fraction),
    //   phz[k][z] = exp(i 2 pi f0 (tau_tx - z / c))
    //   rxd[e][pix] = (r - z) fs / c,  rxp[e][pix] = exp(i 2 pi f0 (r - z) / c),  r - z = dx^2 / (r + z)
    const double L = (c.n_elem - 1) * c.pitch;
    const size_t npix = (size_t)c.nz * c.nu;
    std::vector<float> stx((size_t)c.n_angles * c.nz);
    std::vector<int> sti((size_t)c.n_angles * c.nz);
    std::vector<float2> phz((size_t)c.n_angles * c.nz);
    for (int k = 0; k < c.n_angles; ++k) {
        const double th = c.angles_rad[k];
        for (int l = 0; l < c.nz; ++l) {
            const double z = c.z0 + l * c.dz;
            const double ttx = (z * cos(th) + c.v_ref * sin(th) + 0.5 * L * fabs(sin(th))) / c.c;
            const double sfull = (ttx + z / c.c - c.t_start) * c.fs;
            const double sint = floor(sfull);
            stx[k * c.nz + l] = (float)(sfull - sint);       // fraction in [0, 1)
            sti[k * c.nz + l] = (int)sint;
            double cyc = c.f0 * (ttx - z / c.c);
            cyc -= nearbyint(cyc);
            phz[k * c.nz + l] = make_float2((float)cos(2 * M_PI * cyc), (float)sin(2 * M_PI * cyc));
        }
    }
    std::vector<float> rxd((size_t)c.n_elem * npix);
    std::vector<float2> rxp((size_t)c.n_elem * npix);
    for (int e = 0; e < c.n_elem; ++e) {
        const double ue = (e - 0.5 * (c.n_elem - 1)) * c.pitch;
        for (int l = 0; l < c.nz; ++l) {
            const double z = c.z0 + l * c.dz;
            for (int i = 0; i < c.nu; ++i) {
                const double dx = c.u0 + i * c.du - ue;
                const double drz = dx * dx / (sqrt(dx * dx + z * z) + z);
                const size_t q = (size_t)e * npix + (size_t)l * c.nu + i;
                rxd[q] = (float)(drz * c.fs / c.c);
                double cyc = c.f0 * drz / c.c;
                cyc -= nearbyint(cyc);
                rxp[q] = make_float2((float)cos(2 * M_PI * cyc), (float)sin(2 * M_PI * cyc));
            }
        }
    }
    // DAS windows: for every (transmit, tile, element) the first sample any pixel
    // of the tile reads, from the same FP32 sum s = rxd + stx the kernel forms,
    // and the number of 16-sample chunks from there to the last one it reads,
    // packed as start * 16 + (chunks - 1)
    const int n_tu = cdiv(c.nu, kDasTileU), n_tz = cdiv(c.nz, kDasTileZ), n_tiles = n_tu * n_tz;
    std::vector<int> win((size_t)c.n_angles * n_tiles * c.n_elem);
    int wspan = 0;
    for (int k = 0; k < c.n_angles; ++k)
        for (int tz = 0; tz < n_tz; ++tz)
            for (int tu = 0; tu < n_tu; ++tu)
                for (int e = 0; e < c.n_elem; ++e) {
                    int lo = 1 << 30, hi = -(1 << 30);
                    for (int l = tz * kDasTileZ; l < std::min((tz + 1) * kDasTileZ, c.nz); ++l) {
                        const float sz = stx[k * c.nz + l];
                        const int si = sti[k * c.nz + l];
                        const float *rr = rxd.data() + (size_t)e * npix + (size_t)l * c.nu;
                        for (int i = tu * kDasTileU; i < std::min((tu + 1) * kDasTileU, c.nu); ++i) {
                            const volatile float sv = rr[i] + sz;     // IEEE single-precision sum
                            const int fl = (int)floorf(sv) + si;
                            lo = std::min(lo, fl);
                            hi = std::max(hi, fl);
                        }
                    }
                    const int chunks = cdiv(hi - lo + 1, 16);
                    win[((size_t)k * n_tiles + (tz * n_tu + tu)) * c.n_elem + e] = lo * 16 + (chunks - 1);
                    wspan = std::max(wspan, hi - lo + 1);
                }
    const int das_len = wspan <= 64 ? 64 : (wspan <= 128 ? 128 : 0);
    if (!das_len) {
        char buf[160];
        snprintf(buf, sizeof buf, "delay span of a beamforming tile (%d samples) exceeds the 128-sample window",
                 wspan);
        return fail(ULM_ERR_INVALID_ARG, buf);
    }

    // stage-2 axial taps per (transmit, block): H[d] = sum_m exp(i phi_m) Lambda(d_m - d)
    const int per = cdiv(c.nv, c.n_blocks);
    std::vector<std::vector<std::complex<double>>> acc((size_t)c.n_angles * c.n_blocks);
    std::vector<int2> meta((size_t)c.n_angles * c.n_blocks);
    const int span = 4 * (c.nz + 8);
    int max_taps = 1;
    for (int k = 0; k < c.n_angles; ++k) {
        const double tk = tan(0.5 * c.angles_rad[k]);
        for (int b = 0; b < c.n_blocks; ++b) {
            auto &h = acc[k * c.n_blocks + b];
            h.assign(2 * span + 1, 0.0);
            for (int m = b * per; m < std::min((b + 1) * per, c.nv); ++m) {
                const double dv = c.v0 + m * c.dv - c.v_ref;
                const double d = dv * tk / c.dz;
                const double ph = 4.0 * M_PI * c.f0 * dv * tk / c.c;
                const double fl = floor(d);
                const int n = (int)fl;
                const double fr = d - fl;
                if (n < -span || n + 1 > span) return fail(ULM_ERR_INVALID_ARG, "stage-2 shift out of range");
                const std::complex<double> e = std::polar(1.0, ph);
                h[n + span] += (1.0 - fr) * e;
                h[n + 1 + span] += fr * e;
            }
            int lo = 0, hi = -1;
            for (int q = 0; q <= 2 * span; ++q)
                if (h[q] != 0.0) {
                    if (hi < lo) lo = q;
                    hi = q;
                }
            if (hi < lo) lo = hi = span;        // an empty block: one zero tap
            meta[k * c.n_blocks + b] = make_int2(lo - span, hi - lo + 1);
            max_taps = std::max(max_taps, hi - lo + 1);
        }
    }
    if (max_taps > kFirMaxTaps) return fail(ULM_ERR_INVALID_ARG, "stage-2 shift needs too many taps");
    // stage 2 runs kFirGroup slabs per work-group from one slice tile when the
    // union of their tap ranges fits the tile's halo
    int fir_group = 1;
    if (c.n_blocks >= kFirGroup) {
        int gspan = 0;
        for (int k = 0; k < c.n_angles; ++k)
            for (int b0 = 0; b0 < c.n_blocks; b0 += kFirGroup) {
                int lo = INT32_MAX, hi = INT32_MIN;
                for (int b = b0; b < std::min(b0 + kFirGroup, c.n_blocks); ++b) {
                    const int2 m = meta[k * c.n_blocks + b];
                    lo = std::min(lo, m.x);
                    hi = std::max(hi, m.x + m.y);
                }
                gspan = std::max(gspan, hi - lo);
            }
        if (gspan <= kFirMaxTaps) fir_group = kFirGroup;
    }
    std::vector<float2> taps((size_t)c.n_angles * c.n_blocks * max_taps, make_float2(0.f, 0.f));
    for (int kb = 0; kb < c.n_angles * c.n_blocks; ++kb)
        for (int q = 0; q < meta[kb].y; ++q) {
            const std::complex<double> v = acc[kb][meta[kb].x + q + span];
            taps[(size_t)kb * max_taps + q] = make_float2((float)v.real(), (float)v.imag());
        }

    ulm_ctx *ctx = new (std::nothrow) ulm_ctx();
    if (!ctx) return fail(ULM_ERR_INVALID_ARG, "out of host memory");
    ctx->cfg = c;
    Geometry &g = ctx->geo;
    g.n_elem = c.n_elem;
    g.n_samp = c.n_samp;
    g.n_frames = c.n_frames;
    g.n_angles = c.n_angles;
    g.nu = c.nu;
    g.nz = c.nz;
    g.n_blocks = c.n_blocks;
    g.n_planes = 2 * c.n_blocks;
    g.pitch = (float)c.pitch;
    g.fs_over_c = (float)(c.fs / c.c);
    g.f0_over_c = (float)(c.f0 / c.c);
    g.t_start_fs = (float)(c.t_start * c.fs);
    g.du = (float)c.du;
    g.dz = (float)c.dz;
    g.u0 = (float)c.u0;
    g.z0 = (float)c.z0;
    ctx->tab.n_taps = max_taps;
    ctx->tab.fir_group = fir_group;
    layout_workspace(ctx);

    ctx->tab.das_len = das_len;
    auto cleanup = [&](hipError_t e, const char *where) {
        free_tables(ctx);
        delete ctx;
        return hip_fail(e, where);
    };
    hipError_t e;
    if ((e = hipGetDevice(&ctx->device)) != hipSuccess) return cleanup(e, "hipGetDevice");
    // device address of the library-owned scratch array (ulm_pair_planes_noalloc)
    if ((e = scratch_init(ctx->device)) != hipSuccess) return cleanup(e, "hipGetSymbolAddress(scratch)");
    if ((e = hipMalloc(&ctx->tab.stx, sizeof(float) * stx.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->tab.phz, sizeof(float2) * phz.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->tab.taps, sizeof(float2) * taps.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->tab.tap_meta, sizeof(int2) * meta.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMemcpy(ctx->tab.tap_meta, meta.data(), sizeof(int2) * meta.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMalloc(&ctx->tab.angles, sizeof(double) * ULM_MAX_ANGLES)) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->tab.rxd, sizeof(float) * rxd.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->tab.sti, sizeof(int) * sti.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMemcpy(ctx->tab.sti, sti.data(), sizeof(int) * sti.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMalloc(&ctx->tab.rxp, sizeof(float2) * rxp.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->tab.win, sizeof(int) * win.size())) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMemcpy(ctx->tab.rxd, rxd.data(), sizeof(float) * rxd.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->tab.rxp, rxp.data(), sizeof(float2) * rxp.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->tab.win, win.data(), sizeof(int) * win.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->tab.stx, stx.data(), sizeof(float) * stx.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->tab.phz, phz.data(), sizeof(float2) * phz.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->tab.taps, taps.data(), sizeof(float2) * taps.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->tab.angles, c.angles_rad, sizeof(double) * ULM_MAX_ANGLES, hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    {
        const std::vector<float2> tw = separate_twiddles(c.n_frames);
        if (!tw.empty()) {
            if ((e = hipMalloc(&ctx->tab.sep_tw, sizeof(float2) * tw.size())) != hipSuccess) return cleanup(e, "hipMalloc");
            if ((e = hipMemcpy(ctx->tab.sep_tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice)) != hipSuccess)
                return cleanup(e, "hipMemcpy");
        }
    }
    if (square_grid(c)) {
        // cross projection: column i of the other orientation's volume is its
        // reference slice moved by d = (v_i - v_ref) t_k / dz rows and turned by
        // exp(i 4 pi f0 (v_i - v_ref) t_k / c) (stage 2's shift law)
        std::vector<int> xn((size_t)c.n_angles * c.nu);
        std::vector<float4> xw((size_t)c.n_angles * c.nu);
        for (int k = 0; k < c.n_angles; ++k) {
            const double tk = tan(0.5 * c.angles_rad[k]);
            for (int i = 0; i < c.nu; ++i) {
                const double dv = c.v0 + i * c.dv - c.v_ref;
                const double d = dv * tk / c.dz;
                const double fl = floor(d);
                const double fr = d - fl;
                const double ph = 4.0 * M_PI * c.f0 * dv * tk / c.c;
                const double er = cos(ph), ei = sin(ph);
                xn[(size_t)k * c.nu + i] = (int)fl;
                if (k == 0 && i == 0) ctx->tab.xd_nmin = ctx->tab.xd_nmax = (int)fl;
                ctx->tab.xd_nmin = std::min(ctx->tab.xd_nmin, (int)fl);
                ctx->tab.xd_nmax = std::max(ctx->tab.xd_nmax, (int)fl);
                xw[(size_t)k * c.nu + i] = make_float4((float)((1.0 - fr) * er), (float)((1.0 - fr) * ei),
                                                       (float)(fr * er), (float)(fr * ei));
            }
        }
        if ((e = hipMalloc(&ctx->tab.xd_n, sizeof(int) * xn.size())) != hipSuccess) return cleanup(e, "hipMalloc");
        if ((e = hipMalloc(&ctx->tab.xd_w, sizeof(float4) * xw.size())) != hipSuccess) return cleanup(e, "hipMalloc");
        if ((e = hipMemcpy(ctx->tab.xd_n, xn.data(), sizeof(int) * xn.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return cleanup(e, "hipMemcpy");
        if ((e = hipMemcpy(ctx->tab.xd_w, xw.data(), sizeof(float4) * xw.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return cleanup(e, "hipMemcpy");
    }
    int lds_max = 0;
    if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device)) != hipSuccess)
        return cleanup(e, "hipDeviceGetAttribute");
    if (ncc_lds_bytes(c.nu, (c.ncc_size - 1) / 2) > (size_t)lds_max ||
        (size_t)2 * 8 * c.n_samp * sizeof(float) > (size_t)lds_max) {
        free_tables(ctx);
        delete ctx;
        return fail(ULM_ERR_INVALID_ARG, "plane width or sample count exceeds the device's LDS per work-group");
    }
    for (int i = 0; i < 4; ++i)
        if ((e = hipEventCreate(&ctx->ev[i])) != hipSuccess) return cleanup(e, "hipEventCreate");
    *out = ctx;
    return ULM_OK;
}

extern "C" int32_t ulm_destroy(ulm_ctx_t *ctx) {
    if (!ctx) return ULM_OK;
    free_tables(ctx);
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ctx->ev[i]);
    delete ctx;
    return ULM_OK;
}

extern "C" int32_t ulm_workspace_size(const ulm_ctx_t *ctx, size_t *bytes) {
    if (!ctx || !bytes) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    *bytes = ctx->ws.total;
    return ULM_OK;
}

static int32_t check_ws(const ulm_ctx_t *ctx, void *ws, size_t ws_bytes) {
    if (!ctx) return fail(ULM_ERR_INVALID_ARG, "NULL context");
    if (!ws) return fail(ULM_ERR_INVALID_ARG, "NULL workspace");
    if (ws_bytes < ctx->ws.total) return fail(ULM_ERR_INVALID_ARG, "workspace too small");
    if (((uintptr_t)ws & 255) != 0) return fail(ULM_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    return ULM_OK;
}

extern "C" int32_t rca_beamform_stage1(ulm_ctx_t *ctx, const float *iq, void *ws, size_t ws_bytes,
                                       void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!iq) return fail(ULM_ERR_INVALID_ARG, "NULL iq");
    HIP_TRY(launch_stage1(ctx, (const float2 *)iq, (float2 *)((char *)ws + ctx->ws.slices),
                          (hipStream_t)stream),
            "rca_beamform_stage1");
    return ULM_OK;
}

extern "C" int32_t rca_beamform_stage2(ulm_ctx_t *ctx, float *proj, void *ws, size_t ws_bytes,
                                       void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!proj) return fail(ULM_ERR_INVALID_ARG, "NULL proj");
    HIP_TRY(launch_stage2(ctx, (const float2 *)((char *)ws + ctx->ws.slices), (float2 *)proj,
                          (hipStream_t)stream),
            "rca_beamform_stage2");
    return ULM_OK;
}

extern "C" int32_t rca_beamform_proj(ulm_ctx_t *ctx, const float *iq, float *proj, void *ws,
                                     size_t ws_bytes, void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!iq || !proj) return fail(ULM_ERR_INVALID_ARG, "NULL iq or proj");
    if ((rc = rca_beamform_stage1(ctx, iq, ws, ws_bytes, stream))) return rc;
    return rca_beamform_stage2(ctx, proj, ws, ws_bytes, stream);
}

extern "C" int32_t rca_beamform_cross(ulm_ctx_t *ctx, float *proj_cross, void *ws, size_t ws_bytes,
                                      void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!proj_cross) return fail(ULM_ERR_INVALID_ARG, "NULL cross-projection buffer");
    if (!square_grid(ctx->cfg))
        return fail(ULM_ERR_INVALID_ARG, "the cross projection needs the v grid equal to the u grid");
    if (!cross_supported(ctx->geo, cdiv(ctx->geo.nu, ctx->geo.n_blocks)))
        return fail(ULM_ERR_INVALID_ARG,
                    "cross projection: plane width above 1024 or n_angles x nz x 8 bytes above 64 KiB");
    HIP_TRY(launch_cross(ctx, (const float2 *)((char *)ws + ctx->ws.slices),
                         (float2 *)((char *)ws + ctx->ws.xprof), (float2 *)proj_cross,
                         (hipStream_t)stream),
            "rca_beamform_cross");
    return ULM_OK;
}

extern "C" int32_t ulm_xdoppler(ulm_ctx_t *ctx, const float *native, const float *cross,
                                int32_t window, float *out, void *stream) {
    if (!ctx || !native || !cross || !out) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    if (window < 1 || window > 9 || (window & 1) == 0)
        return fail(ULM_ERR_INVALID_ARG, "window must be odd, in [1, 9]");
    if (out == cross) return fail(ULM_ERR_INVALID_ARG, "out may alias the native stack, not the cross stack");
    HIP_TRY(launch_xdoppler(ctx, (const float2 *)native, (const float2 *)cross, window, (float2 *)out,
                            (hipStream_t)stream),
            "ulm_xdoppler");
    return ULM_OK;
}

extern "C" int32_t svd_clutter_filter(ulm_ctx_t *ctx, float *proj, double *eigvals, void *ws,
                                      size_t ws_bytes, void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!proj) return fail(ULM_ERR_INVALID_ARG, "NULL proj");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_filter(ctx, (float2 *)proj, eigvals, (char *)ws, st), "svd_clutter_filter");
    return ULM_OK;
}

extern "C" int32_t ncc_localize(ulm_ctx_t *ctx, const float *filtered, ulm_loc_t *locs,
                                int32_t capacity, int32_t *count, void *ws, size_t ws_bytes,
                                void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!filtered || !count || capacity < 0 || (capacity > 0 && !locs))
        return fail(ULM_ERR_INVALID_ARG, "NULL filtered/count/locs or negative capacity");
    HIP_TRY(launch_localize(ctx, (const float2 *)filtered, locs, capacity, count, (char *)ws,
                            (hipStream_t)stream),
            "ncc_localize");
    return ULM_OK;
}

// beamform -> filter -> `localize` (a call of the same stream), with the
// optional per-stage timing
template <typename Loc>
static int32_t reconstruct(ulm_ctx_t *ctx, const float *iq, float *proj, double *eigvals, void *ws,
                           size_t ws_bytes, ulm_timing_t *timing, void *stream, Loc localize) {
    hipStream_t st = (hipStream_t)stream;
    int32_t rc;
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[0], st), "hipEventRecord");
    if ((rc = rca_beamform_proj(ctx, iq, proj, ws, ws_bytes, stream))) return rc;
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[1], st), "hipEventRecord");
    if ((rc = svd_clutter_filter(ctx, proj, eigvals, ws, ws_bytes, stream))) return rc;
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[2], st), "hipEventRecord");
    if ((rc = localize())) return rc;
    if (timing) {
        HIP_TRY(hipEventRecord(ctx->ev[3], st), "hipEventRecord");
        HIP_TRY(hipEventSynchronize(ctx->ev[3]), "hipEventSynchronize");
        HIP_TRY(hipEventElapsedTime(&timing->ms_beamform, ctx->ev[0], ctx->ev[1]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&timing->ms_filter, ctx->ev[1], ctx->ev[2]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&timing->ms_localize, ctx->ev[2], ctx->ev[3]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&timing->ms_total, ctx->ev[0], ctx->ev[3]), "hipEventElapsedTime");
    }
    return ULM_OK;
}

extern "C" int32_t ulm_reconstruct_ensemble(ulm_ctx_t *ctx, const float *iq, float *proj,
                                            double *eigvals, ulm_loc_t *locs, int32_t capacity,
                                            int32_t *count, void *ws, size_t ws_bytes,
                                            ulm_timing_t *timing, void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!iq || !proj || !count || capacity < 0 || (capacity > 0 && !locs))
        return fail(ULM_ERR_INVALID_ARG, "NULL argument or negative capacity");
    return reconstruct(ctx, iq, proj, eigvals, ws, ws_bytes, timing, stream, [&] {
        return ncc_localize(ctx, proj, locs, capacity, count, ws, ws_bytes, stream);
    });
}

extern "C" int32_t ulm_check_status(ulm_ctx_t *ctx, void *ws, const int32_t *count,
                                    int32_t capacity, void *stream) {
    if (!ctx || !ws) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    int status = 0;
    HIP_TRY(hipMemcpy(&status, (char *)ws + ctx->ws.status, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
    if (status & kStatusNumeric) return fail(ULM_ERR_NUMERIC, "non-finite covariance: plane left unfiltered");
    if (status & kStatusBarrier) return fail(ULM_ERR_NUMERIC, "eigensolver wait timed out: filter result invalid");
    if (status & kStatusCnnRow) return fail(ULM_ERR_OVERFLOW, "a CNN decode row held more peaks than its staging slot");
    if (count && capacity >= 0) {
        int n = 0;
        HIP_TRY(hipMemcpy(&n, count, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
        if (n > capacity) return fail(ULM_ERR_OVERFLOW, "more localisations than capacity");
    }
    return ULM_OK;
}

extern "C" int32_t ulm_sim_channel_data(ulm_ctx_t *ctx, const double *pos, const double *amp,
                                        int32_t n_scat, uint64_t noise_seed, double noise_sigma,
                                        float *iq, void *stream) {
    if (!ctx || !iq || n_scat < 0 || (n_scat > 0 && (!pos || !amp)) || !(noise_sigma >= 0))
        return fail(ULM_ERR_INVALID_ARG, "bad simulator argument");
    HIP_TRY(launch_sim(ctx, pos, amp, n_scat, noise_seed, noise_sigma, iq,
                       ctx->tab.angles, (hipStream_t)stream),
            "ulm_sim_channel_data");
    return ULM_OK;
}

extern "C" int32_t ulm_density_accumulate(ulm_ctx_t *ctx, const ulm_loc_t *locs,
                                          const int32_t *count, int32_t capacity,
                                          int32_t upsample, uint32_t *density, void *stream) {
    if (!ctx || !count || !density || capacity < 0 || upsample < 1 || upsample > 16 ||
        (capacity > 0 && !locs))
        return fail(ULM_ERR_INVALID_ARG, "bad density argument");
    HIP_TRY(launch_density(ctx, locs, count, capacity, upsample, density, (hipStream_t)stream),
            "ulm_density_accumulate");
    return ULM_OK;
}

// ---------------------------------------------------------------- learned localiser

static int32_t cnn_dims(int32_t batch, int32_t nz, int32_t nu, int32_t precision) {
    if (batch < 1 || nz < 1 || nu < 1) return fail(ULM_ERR_INVALID_ARG, "batch, nz, nu must be >= 1");
    if ((int64_t)batch * nz * nu > (int64_t)1 << 26)
        return fail(ULM_ERR_INVALID_ARG, "batch * nz * nu above 2^26 pixels");
    if ((int64_t)nz * 8 * nu * 8 > INT32_MAX) return fail(ULM_ERR_INVALID_ARG, "image too large");
    if (precision != ULM_CNN_BF16 && precision != ULM_CNN_FP32)
        return fail(ULM_ERR_INVALID_ARG, "precision must be ULM_CNN_BF16 or ULM_CNN_FP32");
    return ULM_OK;
}

static int32_t check_cws(void *cws, size_t have, size_t need) {
    if (!cws) return fail(ULM_ERR_INVALID_ARG, "NULL CNN workspace");
    if (have < need) return fail(ULM_ERR_INVALID_ARG, "CNN workspace too small");
    if (((uintptr_t)cws & 255) != 0) return fail(ULM_ERR_INVALID_ARG, "CNN workspace not 256-byte aligned");
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_workspace_size(int32_t batch, int32_t nz, int32_t nu, int32_t precision,
                                          int32_t train, size_t *bytes) {
    int32_t rc = cnn_dims(batch, nz, nu, precision);
    if (rc) return rc;
    if (!bytes) return fail(ULM_ERR_INVALID_ARG, "NULL bytes");
    *bytes = cnn_workspace_bytes(batch, nz, nu, precision == ULM_CNN_FP32, train != 0);
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_localize_workspace_size(const ulm_ctx_t *ctx, int32_t batch,
                                                   int32_t precision, size_t *bytes) {
    if (!ctx || !bytes) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    int32_t rc = cnn_dims(batch, ctx->geo.nz, ctx->geo.nu, precision);
    if (rc) return rc;
    const int n_img = ctx->geo.n_planes * ctx->geo.n_frames;
    *bytes = cnn_loc_workspace_bytes(batch, ctx->geo.nz, ctx->geo.nu, n_img, precision == ULM_CNN_FP32);
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_images(ulm_ctx_t *ctx, const float *filtered, float *images, void *ws,
                                  size_t ws_bytes, void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!filtered || !images) return fail(ULM_ERR_INVALID_ARG, "NULL filtered/images");
    const Geometry &g = ctx->geo;
    const int n_img = g.n_planes * g.n_frames, npix = g.nz * g.nu;
    hipStream_t st = (hipStream_t)stream;
    float *fmax = (float *)((char *)ws + ctx->ws.fmax);
    HIP_TRY(launch_frame_max((const float2 *)filtered, fmax, n_img, npix, st), "ulm_cnn_images");
    HIP_TRY(cnn_images((const float2 *)filtered, fmax, images, npix, 0, n_img, st), "ulm_cnn_images");
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_forward(const float *params, const float *images, int32_t batch,
                                   int32_t nz, int32_t nu, int32_t precision, float *heat,
                                   void *cnn_ws, size_t cnn_ws_bytes, void *stream) {
    int32_t rc = cnn_dims(batch, nz, nu, precision);
    if (rc) return rc;
    if (!params || !images || !heat) return fail(ULM_ERR_INVALID_ARG, "NULL params/images/heat");
    const bool fp32 = precision == ULM_CNN_FP32;
    if ((rc = check_cws(cnn_ws, cnn_ws_bytes, cnn_workspace_bytes(batch, nz, nu, fp32, false)))) return rc;
    HIP_TRY(cnn_forward_heat(params, images, heat, batch, nz, nu, fp32, (char *)cnn_ws,
                             (hipStream_t)stream),
            "ulm_cnn_forward");
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_gradients(const float *params, const float *images, int32_t batch,
                                     int32_t nz, int32_t nu, const float *mb_zu,
                                     const int32_t *mb_img, int32_t n_mb, int32_t precision,
                                     float *grad, float *loss, void *cnn_ws, size_t cnn_ws_bytes,
                                     void *stream) {
    int32_t rc = cnn_dims(batch, nz, nu, precision);
    if (rc) return rc;
    if (!params || !images || !grad || !loss || n_mb < 0 || (n_mb > 0 && (!mb_zu || !mb_img)))
        return fail(ULM_ERR_INVALID_ARG, "NULL argument or negative n_mb");
    const bool fp32 = precision == ULM_CNN_FP32;
    if ((rc = check_cws(cnn_ws, cnn_ws_bytes, cnn_workspace_bytes(batch, nz, nu, fp32, true)))) return rc;
    HIP_TRY(cnn_gradients(params, images, mb_zu, mb_img, n_mb, batch, nz, nu, fp32, grad, loss,
                          (char *)cnn_ws, (hipStream_t)stream),
            "ulm_cnn_gradients");
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_train_step(float *params, float *adam_m, float *adam_v, int32_t step,
                                      float lr, const float *images, int32_t batch, int32_t nz,
                                      int32_t nu, const float *mb_zu, const int32_t *mb_img,
                                      int32_t n_mb, int32_t precision, float *loss, void *cnn_ws,
                                      size_t cnn_ws_bytes, void *stream) {
    if (!adam_m || !adam_v || step < 1 || !(lr >= 0.f))
        return fail(ULM_ERR_INVALID_ARG, "NULL Adam state, step < 1 or bad lr");
    const bool fp32 = precision == ULM_CNN_FP32;
    int32_t rc = cnn_dims(batch, nz, nu, precision);
    if (rc) return rc;
    if ((rc = check_cws(cnn_ws, cnn_ws_bytes, cnn_workspace_bytes(batch, nz, nu, fp32, true)))) return rc;
    float *grad = cnn_ws_grad(batch, nz, nu, fp32, (char *)cnn_ws);
    if ((rc = ulm_cnn_gradients(params, images, batch, nz, nu, mb_zu, mb_img, n_mb, precision, grad,
                                loss, cnn_ws, cnn_ws_bytes, stream)))
        return rc;
    HIP_TRY(cnn_adam(params, adam_m, adam_v, grad, step, lr, (hipStream_t)stream), "ulm_cnn_train_step");
    return ULM_OK;
}

extern "C" int32_t ulm_cnn_localize(ulm_ctx_t *ctx, const float *params, const float *filtered,
                                    float threshold, int32_t batch, int32_t precision,
                                    ulm_loc_t *locs, int32_t capacity, int32_t *count, void *ws,
                                    size_t ws_bytes, void *cnn_ws, size_t cnn_ws_bytes,
                                    void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    const Geometry &g = ctx->geo;
    if ((rc = cnn_dims(batch, g.nz, g.nu, precision))) return rc;
    if (!params || !filtered || !count || capacity < 0 || (capacity > 0 && !locs))
        return fail(ULM_ERR_INVALID_ARG, "NULL params/filtered/count/locs or negative capacity");
    if (!(threshold > -1e30f && threshold < 1e30f)) return fail(ULM_ERR_INVALID_ARG, "threshold not finite");
    const bool fp32 = precision == ULM_CNN_FP32;
    const int n_img = g.n_planes * g.n_frames;
    if ((rc = check_cws(cnn_ws, cnn_ws_bytes, cnn_loc_workspace_bytes(batch, g.nz, g.nu, n_img, fp32))))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    float *fmax = (float *)((char *)ws + ctx->ws.fmax);
    int *status = (int *)((char *)ws + ctx->ws.status);
    HIP_TRY(launch_frame_max((const float2 *)filtered, fmax, n_img, g.nz * g.nu, st), "ulm_cnn_localize");
    HIP_TRY(cnn_localize(params, (const float2 *)filtered, fmax, threshold, n_img, g.n_frames, g.nz,
                         g.nu, batch, fp32, locs, capacity, count, status, (char *)cnn_ws, st),
            "ulm_cnn_localize");
    return ULM_OK;
}

extern "C" int32_t ulm_reconstruct_ensemble_cnn(ulm_ctx_t *ctx, const float *iq, float *proj,
                                                double *eigvals, const float *params, float threshold,
                                                int32_t batch, int32_t precision, ulm_loc_t *locs,
                                                int32_t capacity, int32_t *count, void *ws,
                                                size_t ws_bytes, void *cnn_ws, size_t cnn_ws_bytes,
                                                ulm_timing_t *timing, void *stream) {
    int32_t rc = check_ws(ctx, ws, ws_bytes);
    if (rc) return rc;
    if (!iq || !proj || !params || !count || capacity < 0 || (capacity > 0 && !locs))
        return fail(ULM_ERR_INVALID_ARG, "NULL argument or negative capacity");
    // the CNN's own checks, before any work is queued
    if ((rc = cnn_dims(batch, ctx->geo.nz, ctx->geo.nu, precision))) return rc;
    if (!(threshold > -1e30f && threshold < 1e30f)) return fail(ULM_ERR_INVALID_ARG, "threshold not finite");
    const int n_img = ctx->geo.n_planes * ctx->geo.n_frames;
    if ((rc = check_cws(cnn_ws, cnn_ws_bytes,
                        cnn_loc_workspace_bytes(batch, ctx->geo.nz, ctx->geo.nu, n_img, precision == ULM_CNN_FP32))))
        return rc;
    return reconstruct(ctx, iq, proj, eigvals, ws, ws_bytes, timing, stream, [&] {
        return ulm_cnn_localize(ctx, params, proj, threshold, batch, precision, locs, capacity, count, ws,
                                ws_bytes, cnn_ws, cnn_ws_bytes, stream);
    });
}

// ---------------------------------------------------------------- plane pairing

extern "C" int32_t ulm_pair_workspace_size(const ulm_ctx_t *ctx, int32_t capacity, size_t *bytes) {
    if (!ctx || !bytes || capacity < 0) return fail(ULM_ERR_INVALID_ARG, "NULL argument or negative capacity");
    *bytes = pair_workspace_bytes(ctx->geo.n_planes, ctx->geo.n_frames, std::max(capacity, 1));
    return ULM_OK;
}

extern "C" int32_t ulm_pair_planes(ulm_ctx_t *ctx, const ulm_loc_t *locs, const int32_t *count,
                                   int32_t capacity, ulm_loc3d_t *out, int32_t out_capacity,
                                   int32_t *out_count, void *pws, size_t pws_bytes, void *stream) {
    if (!ctx || !count || !out_count || capacity < 0 || out_capacity < 0 ||
        (capacity > 0 && !locs) || (out_capacity > 0 && !out))
        return fail(ULM_ERR_INVALID_ARG, "NULL argument or negative capacity");
    if (!pws || pws_bytes < pair_workspace_bytes(ctx->geo.n_planes, ctx->geo.n_frames, std::max(capacity, 1)))
        return fail(ULM_ERR_INVALID_ARG, "pairing workspace missing or too small");
    if (((uintptr_t)pws & 255) != 0) return fail(ULM_ERR_INVALID_ARG, "pairing workspace not 256-byte aligned");
    if (((uintptr_t)locs & 15) != 0) return fail(ULM_ERR_INVALID_ARG, "localisation list not 16-byte aligned");
    HIP_TRY(launch_pairing(ctx, locs, count, capacity, out, out_capacity, out_count, (char *)pws,
                           (hipStream_t)stream),
            "ulm_pair_planes");
    return ULM_OK;
}

extern "C" int32_t ulm_pair_planes_noalloc(ulm_ctx_t *ctx, const ulm_loc_t *locs,
                                           const int32_t *count, int32_t capacity,
                                           ulm_loc3d_t *out, int32_t out_capacity,
                                           int32_t *out_count, void *stream) {
    if (!ctx || !count || !out_count || capacity < 0 || out_capacity < 0 ||
        (capacity > 0 && !locs) || (out_capacity > 0 && !out))
        return fail(ULM_ERR_INVALID_ARG, "NULL argument or negative capacity");
    const size_t need = pair_workspace_bytes(ctx->geo.n_planes, ctx->geo.n_frames, std::max(capacity, 1));
    if (need > (size_t)ULM_NOALLOC_SCRATCH_BYTES)
        return fail(ULM_ERR_INVALID_ARG,
                    "capacity too large for the library scratch array: the pairing needs " +
                        std::to_string(need) + " bytes, the array holds " +
                        std::to_string((size_t)ULM_NOALLOC_SCRATCH_BYTES));
    if (((uintptr_t)locs & 15) != 0) return fail(ULM_ERR_INVALID_ARG, "localisation list not 16-byte aligned");
    char *pws = (char *)scratch_ptr(ctx->device);
    if (!pws) return fail(ULM_ERR_HIP, "library scratch array has no device address on this device");
    HIP_TRY(launch_pairing(ctx, locs, count, capacity, out, out_capacity, out_count, pws,
                           (hipStream_t)stream),
            "ulm_pair_planes_noalloc");
    return ULM_OK;
}

// ---------------------------------------------------------------- motion estimation

extern "C" int32_t ulm_slices_offset(const ulm_ctx_t *ctx, size_t *offset) {
    if (!ctx || !offset) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    *offset = ctx->ws.slices;
    return ULM_OK;
}

static int32_t check_lag(const ulm_ctx_t *ctx, int32_t max_lag) {
    const Geometry &g = ctx->geo;
    if (max_lag < 1 || max_lag > 10) return fail(ULM_ERR_INVALID_ARG, "max_lag must lie in [1, 10]");
    if (2 * max_lag + 1 > g.nz || 2 * max_lag + 1 > g.nu)
        return fail(ULM_ERR_INVALID_ARG, "lag window larger than the slice");
    if (motion_lds_bytes(g, max_lag) == 0)
        return fail(ULM_ERR_INVALID_ARG, "slice too wide for the motion kernel's LDS band");
    return ULM_OK;
}

extern "C" int32_t ulm_motion_workspace_size(const ulm_ctx_t *ctx, int32_t max_lag, size_t *bytes) {
    if (!ctx || !bytes) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    const int32_t r = check_lag(ctx, max_lag);
    if (r != ULM_OK) return r;
    *bytes = motion_workspace_bytes(ctx->geo, max_lag);
    return ULM_OK;
}

extern "C" int32_t ulm_motion_estimate(ulm_ctx_t *ctx, const float *slices, int32_t ref_frame,
                                       int32_t max_lag, float *disp, float *motion, void *mws,
                                       size_t mws_bytes, void *stream) {
    if (!ctx || !slices || !disp || !motion || !mws) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    const int32_t r = check_lag(ctx, max_lag);
    if (r != ULM_OK) return r;
    if (ref_frame < 0 || ref_frame >= ctx->geo.n_frames)
        return fail(ULM_ERR_INVALID_ARG, "reference frame outside the ensemble");
    if (mws_bytes < motion_workspace_bytes(ctx->geo, max_lag))
        return fail(ULM_ERR_INVALID_ARG, "motion workspace too small");
    if (((uintptr_t)mws & 255) != 0) return fail(ULM_ERR_INVALID_ARG, "motion workspace not 256-byte aligned");
    HIP_TRY(launch_motion(ctx, (const float2 *)slices, ref_frame, max_lag, disp, motion, (char *)mws,
                          (hipStream_t)stream),
            "ulm_motion_estimate");
    return ULM_OK;
}

// ---------------------------------------------------------------- MB separation

extern "C" int32_t ulm_separate(ulm_ctx_t *ctx, const float *filtered, int32_t n_speed,
                                float *subsets, void *stream) {
    if (!ctx || !filtered || !subsets) return fail(ULM_ERR_INVALID_ARG, "NULL argument");
    if (n_speed < 1 || n_speed > 8) return fail(ULM_ERR_INVALID_ARG, "n_speed must lie in [1, 8]");
    if (!separate_supported(ctx->geo.n_frames))
        return fail(ULM_ERR_INVALID_ARG,
                    "separation needs 2 <= frames <= 512 with no prime factor above 7");
    HIP_TRY(launch_separate(ctx, (const float2 *)filtered, n_speed, (float2 *)subsets,
                            (hipStream_t)stream),
            "ulm_separate");
    return ULM_OK;
}
