/*
 * ulmproj: projection-based RCA ULM reconstruction on AMD MI355X (gfx950).
 *
 * C ABI of libulmproj.so.  Plain C types only: buffers are raw pointers,
 * sizes are integers, the stream is an opaque hipStream_t passed as void*.
 *
 * Conventions for every entry point
 *   - SI units (m, s, Hz, rad).  Complex values are interleaved float pairs
 *     (re, im) ("c64") or double pairs ("c128"); arrays are row-major with the
 *     last index fastest.
 *   - Device buffers are owned by the caller (allocated on the device that was
 *     current at ulm_create).  The context owns only its small tables.
 *   - The workspace `ws` (ws_bytes >= ulm_workspace_size, 256-byte aligned)
 *     is caller-owned device memory.  Zero-fill it once after allocating it;
 *     its contents between calls are otherwise unspecified, except that
 *     ulm_check_status reads the status word the last call left there.
 *   - Calls are asynchronous on `stream` (NULL = the default stream); results
 *     are valid once the caller synchronises that stream.  No entry point
 *     allocates memory, and none synchronises the stream except
 *     ulm_check_status.
 *   - Every entry point returns ULM_OK (0) or a negative error code;
 *     ulm_last_error() returns a thread-local message for the last error.
 *   - Two calls that share a workspace must not overlap in time.
 *
 * The method (paper: "Fast 3D Ultrasound Localization Microscopy via
 * Projection-based Processing Framework"):
 *   Section II-A1  two-stage beamforming: stage-1 reference slice per transmit,
 *                  stage-2 extrapolation along the transmit direction with a
 *                  rigid axial shift, coherent compounding;
 *   Section II-A4  sub-block sum projection onto x-z / y-z planes;
 *   Section II-A2  eigen-based SVD clutter filter: covariance of the Casorati
 *                  matrix, eigendecomposition, projection removal;
 *   Section II-A4  NCC with a Gaussian PSF (separable 1D correlations, Fig. 1g),
 *                  maximum-intensity threshold, sub-pixel regional peaks;
 *   Section IV     learned localisation as the alternative to NCC (ulm_cnn_*).
 */
#ifndef ULMPROJ_H
#define ULMPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ULM_OK                   0
#define ULM_ERR_INVALID_ARG     -1   /* bad pointer, size or configuration        */
#define ULM_ERR_HIP             -2   /* a HIP runtime call failed                 */
#define ULM_ERR_OVERFLOW        -3   /* more localisations than `capacity`        */
#define ULM_ERR_NUMERIC         -4   /* non-finite input to the clutter filter    */
#define ULM_ERR_NOT_IMPLEMENTED -5

#define ULM_MAX_ANGLES 32

/* precision of the Casorati Gram and the clutter removal */
#define ULM_PREC_FP64GRAM 0   /* plain path: FP32 data, Gram and removal accumulated in FP64 */
#define ULM_PREC_BF16X3   1   /* Gram and removal on BF16 MFMA: every operand split into three
                                 BF16 terms (hi, mid, lo), the six products of term orders
                                 below three accumulated in FP32 per 16-pixel (Gram) or
                                 8-frame (removal) K-step, those sums added in FP64        */

typedef struct ulm_config {
    /* probe: n_elem row elements and n_elem column elements */
    int32_t n_elem;
    int32_t n_samp;       /* IQ samples per channel (at least 5)             */
    int32_t n_frames;     /* frames (volumes) per ensemble                   */
    int32_t n_angles;     /* plane-wave angles per orientation (<= 32)       */
    double  pitch;        /* element pitch, m                                */
    double  c;            /* speed of sound, m/s                             */
    double  f0;           /* centre frequency, Hz                            */
    double  fs;           /* IQ sampling rate, Hz                            */
    double  t_start;      /* time of IQ sample 0 after the firing, s         */
    double  bandwidth;    /* fractional -6 dB bandwidth (simulator pulse)    */
    double  angles_rad[ULM_MAX_ANGLES];
    /* projection-plane grid; pixel centres u0 + i*du, z0 + l*dz, v0 + m*dv */
    int32_t nu, nz, nv, n_blocks;
    double  du, dz, u0, z0, dv, v0;
    double  v_ref;        /* stage-1 reference slice position on v           */
    /* clutter filter and localisation */
    int32_t svd_cutoff;   /* removed modes, 0 <= c <= min(32, n_frames)     */
    int32_t ncc_size;     /* odd template size, 3..15                        */
    int32_t precision;    /* ULM_PREC_*                                      */
    int32_t reserved;
    double  sigma_u, sigma_z;   /* template sigmas, pixels                   */
    double  tau_ncc;            /* NCC threshold                             */
    double  alpha;              /* intensity threshold / frame maximum       */
} ulm_config_t;

/* One localisation.  plane = orientation * n_blocks + block; positions are in
 * pixel units of the plane grid (pixel centres at integers). */
typedef struct ulm_loc {
    int32_t plane;
    int32_t frame;
    int32_t iz, iu;       /* integer peak pixel                              */
    float   z, u;         /* sub-pixel position                              */
    float   ncc;          /* NCC at the peak                                 */
    float   intensity;    /* envelope at the peak                            */
} ulm_loc_t;

/* A 3D localisation paired from one XZ and one YZ localisation of a frame. */
typedef struct ulm_loc3d {
    int32_t frame;
    float   x, y, z;          /* plane pixel units: x of the XZ record, y of the YZ record, mean z */
    float   i_xz, i_yz;       /* the two records' intensities                      */
    int32_t idx_xz, idx_yz;   /* their indices in the input list                   */
} ulm_loc3d_t;

typedef struct ulm_timing {
    float ms_beamform, ms_filter, ms_localize, ms_total;
} ulm_timing_t;

typedef struct ulm_ctx ulm_ctx_t;

/* Thread-local message for the last error returned on this thread. */
const char *ulm_last_error(void);

/*
 * Validate `cfg`, build the per-geometry tables (stage-2 axial taps, per-depth
 * transmit delays and phases, NCC template taps) on the current device and
 * return a context.  Errors: INVALID_ARG (bad configuration, including a
 * geometry whose delay span does not fit the beamformer's sample window), HIP.
 */
int32_t ulm_create(const ulm_config_t *cfg, ulm_ctx_t **out);
int32_t ulm_destroy(ulm_ctx_t *ctx);

/* Bytes of device workspace every call below needs. */
int32_t ulm_workspace_size(const ulm_ctx_t *ctx, size_t *bytes);

/*
 * Two-stage beamforming straight to projection planes (Section II-A1 and the
 * sub-block projection of Section II-A4).
 *   iq   [F][2][K][Nc][Ns] c64, device: IQ channel data; orientation 0 = RC
 *        (transmit rows, receive columns: x-z plane), 1 = CR (y-z plane).
 *   proj [2][B][F][Nz][Nu] c64, device, written:
 *        P_{o,b}(u,z) = sum_k sum_{m in block b} S_k^lin(u, z + (v_m - v_ref) t_k)
 *                       * exp(i 4 pi f0 (v_m - v_ref) t_k / c),  t_k = tan(theta_k / 2),
 *        S_k(u,z) = sum_e IQ^lin_{k,e}((tau - t_start) fs) exp(i 2 pi f0 (tau - 2z/c)),
 *        tau = tau_tx(v_ref, z; theta_k) + tau_rx(u, z; e).
 * Errors: INVALID_ARG (NULL pointer, ws too small), HIP.
 */
int32_t rca_beamform_proj(ulm_ctx_t *ctx, const float *iq, float *proj, void *ws,
                          size_t ws_bytes, void *stream);

/*
 * The two halves of rca_beamform_proj, for callers that time or overlap them.
 * rca_beamform_stage1 writes the stage-1 reference slices
 *   S[o][k][f][z][u] (c64) into the workspace;
 * rca_beamform_stage2 reads them from the same workspace and writes `proj`
 * (stage-2 extrapolation, compounding and slab projection as an axial FIR).
 * Errors: INVALID_ARG, HIP.
 */
int32_t rca_beamform_stage1(ulm_ctx_t *ctx, const float *iq, void *ws, size_t ws_bytes,
                            void *stream);
int32_t rca_beamform_stage2(ulm_ctx_t *ctx, float *proj, void *ws, size_t ws_bytes, void *stream);

/*
 * Cross projections for XDoppler (Section II-A4: beamforming and filtering run
 * on the RC and CR volumes separately, and the filtered RC and CR stacks are
 * cross-correlated before localisation).  Both orientations' volumes share one
 * voxel grid, so plane (o, b) also receives the OTHER orientation o' = 1 - o's
 * compounded volume, sum-projected over slab b onto plane o:
 *   Q_{o,b}(v_i, z) = sum_k sum_{u in block b} S^{o'}_k^lin(u, z + (v_i - v_ref) t_k)
 *                     * exp(i 4 pi f0 (v_i - v_ref) t_k / c),   t_k = tan(theta_k / 2),
 * i.e. the plane's lateral column i is the other orientation's slice v_i.
 * Reads the stage-1 slices that rca_beamform_stage1 left in `ws`.
 *   proj_cross [2][B][F][Nz][Nu] c64, device, written.
 * Needs nv == nu, dv == du and v0 == u0, nu <= 1024 and
 * n_angles * nz * 8 <= 65536 (the transmits' slab profiles of a frame in LDS).
 * Errors: INVALID_ARG (grid, NULL pointer, ws too small), HIP.
 */
int32_t rca_beamform_cross(ulm_ctx_t *ctx, float *proj_cross, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * XDoppler image (Section II-A4: cross-correlation of the filtered RC and CR
 * stacks with a window of `window` frames, 3 in the paper):
 *   X_f = sum_{t = f - h .. f + h, 0 <= t < F} native_t * conj(cross_t),  h = (window - 1) / 2,
 *   out[o][b][f][z][u] = (sqrt(|X_f|), 0)
 * sqrt(|X|) is, for one microbubble, the geometric mean of its two
 * orientations' amplitudes, so the localisers' template applies unchanged;
 * ncc_localize and ulm_cnn_localize take `out` as their filtered planes.
 *   native, cross [2][B][F][Nz][Nu] c64, device: the filtered projections and
 *                 cross projections (svd_clutter_filter on each).
 *   out           [2][B][F][Nz][Nu] c64, device; may be `native` itself (in
 *                 place), must not overlap `cross`.
 *   window        odd, in [1, 9].
 * Errors: INVALID_ARG, HIP.
 */
int32_t ulm_xdoppler(ulm_ctx_t *ctx, const float *native, const float *cross, int32_t window,
                     float *out, void *stream);

/*
 * Eigen-based SVD clutter filter of every plane (Section II-A2), in place.
 *   proj    [2][B][F][Nz*Nu] c64, device, in/out.  Each plane's Casorati matrix
 *           I (pixels x frames) becomes I - (I V_c) V_c^H, V_c the eigenvectors of
 *           the svd_cutoff largest eigenvalues of C = I^H I (FP64 eigensolver).
 *   eigvals [2][B][F] f64, device, may be NULL: eigenvalues of C, descending.
 * The context's precision selects how C and I V_c, (I V_c) V_c^H are formed:
 * ULM_PREC_FP64GRAM on FP64 MFMA / FP64 FMAs, ULM_PREC_BF16X3 on BF16 MFMA with
 * three-term split operands (see above); the eigensolver is FP64 in both.
 * A plane with a non-finite covariance is left unfiltered and flags the status
 * word (see ulm_check_status).  Errors: INVALID_ARG, HIP.
 */
int32_t svd_clutter_filter(ulm_ctx_t *ctx, float *proj, double *eigvals, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * NCC localisation (Section II-A4) on filtered planes.
 *   filtered [2][B][F][Nz][Nu] c64, device.
 *   locs     [capacity] ulm_loc_t, device: the first min(total, capacity)
 *            detections sorted by (plane, frame, iz, iu).
 *   count    int32, device: total number of detections (may exceed capacity;
 *            ulm_check_status then returns ULM_ERR_OVERFLOW).
 * Detection: NCC >= tau_ncc, envelope >= alpha * frame maximum, NCC above the
 * 3x3 neighbours earlier in raster order and not below the later ones;
 * sub-pixel offsets by a 3-point Gaussian fit per axis (parabolic when a value
 * is <= 0), clamped to +-0.5.  Errors: INVALID_ARG, HIP.
 */
int32_t ncc_localize(ulm_ctx_t *ctx, const float *filtered, ulm_loc_t *locs, int32_t capacity,
                     int32_t *count, void *ws, size_t ws_bytes, void *stream);

/*
 * The whole path on one ensemble: rca_beamform_proj -> svd_clutter_filter ->
 * ncc_localize.  `proj` receives the filtered planes.  `timing` (host, may be
 * NULL) receives per-stage milliseconds; a non-NULL `timing` synchronises the
 * stream at the end of the call.
 */
int32_t ulm_reconstruct_ensemble(ulm_ctx_t *ctx, const float *iq, float *proj,
                                 double *eigvals, ulm_loc_t *locs, int32_t capacity,
                                 int32_t *count, void *ws, size_t ws_bytes,
                                 ulm_timing_t *timing, void *stream);

/*
 * Synchronise `stream`, then report the status the last svd_clutter_filter /
 * ncc_localize call left in `ws`: ULM_OK, ULM_ERR_NUMERIC (a plane was not
 * filtered) or ULM_ERR_OVERFLOW (count > capacity).  `capacity` is the value
 * passed to the last ncc_localize (or -1 to skip that check); `count` is that
 * call's device counter (may be NULL).
 */
int32_t ulm_check_status(ulm_ctx_t *ctx, void *ws, const int32_t *count, int32_t capacity,
                         void *stream);

/*
 * Forward model of the channel data (input generator; not part of the timed
 * path).  For every frame f, orientation o, angle k, element e and sample s:
 *   IQ = sum_q amp_q exp(-(t_s - tau_q)^2 / (2 sigma_t^2)) exp(-i 2 pi f0 tau_q) + n
 *   sigma_t = sqrt(2 ln 2) / (pi bandwidth f0); the Gaussian is truncated where
 *   it falls below 1e-9; n = Philox4x32-10 / Box-Muller complex noise of rms
 *   noise_sigma keyed by noise_seed and the sample's flat index.
 *   pos [F][S][3] f64, device: scatterer (x, y, z) per frame.
 *   amp [S] c128, device.   iq [F][2][K][Nc][Ns] c64, device, written.
 * Scatterers are accumulated with LDS float atomics: results agree with an
 * exact sum to ~1e-7 but are not bitwise reproducible.
 */
int32_t ulm_sim_channel_data(ulm_ctx_t *ctx, const double *pos, const double *amp,
                             int32_t n_scat, uint64_t noise_seed, double noise_sigma,
                             float *iq, void *stream);

/*
 * Accumulate localisations into per-plane density maps on a grid `upsample`
 * times finer than the planes (pixel i covers [i - 0.5, i + 0.5); fine bin
 * floor((x + 0.5) * upsample)); out-of-grid records are skipped.
 *   locs [n] ulm_loc_t device (n read from the device `count`, clipped to
 *   capacity); density [2*B][Nz*up][Nu*up] uint32, device, incremented.
 */
int32_t ulm_density_accumulate(ulm_ctx_t *ctx, const ulm_loc_t *locs, const int32_t *count,
                               int32_t capacity, int32_t upsample, uint32_t *density,
                               void *stream);

/* Workspace bytes for ulm_pair_planes on an input list of `capacity` records. */
int32_t ulm_pair_workspace_size(const ulm_ctx_t *ctx, int32_t capacity, size_t *bytes);

/*
 * Projection-based 3D localisation (Section II-A4): pair the localisations of
 * the two orthogonal planes of each frame.  An XZ record i (orientation 0) and a
 * YZ record j (orientation 1) of the same frame are candidates when
 * |z_i - z_j| <= 1 (one voxel axially) and I_i / I_j lies in [0.9, 1.11]
 * (intensities = the records' envelope values); with B slabs, j's y must lie in
 * i's slab and i's x in j's slab.  A pair is kept when each is the other's
 * candidate closest to a unit ratio, max(I_i/I_j, I_j/I_i) (ties to the smaller
 * index); its 3D position is (x_i, y_j, (z_i + z_j) / 2).
 *   locs   [capacity] ulm_loc_t, device, 16-byte aligned, sorted by (plane,
 *          frame) as the localisers write them; the first min(*count, capacity)
 *          are used.
 *   out    [out_capacity] ulm_loc3d_t, device: pairs sorted by (frame, idx_xz);
 *   out_count int32, device: total pairs (may exceed out_capacity; then
 *          ulm_check_status(ctx, ws, out_count, out_capacity) returns OVERFLOW).
 *   pws    workspace of at least ulm_pair_workspace_size(ctx, capacity) bytes.
 * Errors: INVALID_ARG, HIP.
 */
int32_t ulm_pair_planes(ulm_ctx_t *ctx, const ulm_loc_t *locs, const int32_t *count,
                        int32_t capacity, ulm_loc3d_t *out, int32_t out_capacity,
                        int32_t *out_count, void *pws, size_t pws_bytes, void *stream);

/* Size of the library-owned device scratch array used by
 * ulm_pair_planes_noalloc (one array per device). */
#define ULM_NOALLOC_SCRATCH_BYTES (32u << 20)

/*
 * ulm_pair_planes without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * ulm_pair_planes minus `pws`: the workspace lives in a fixed library-owned
 * device array of ULM_NOALLOC_SCRATCH_BYTES per device, whose address
 * ulm_create looks up (once per device).  The call allocates nothing.
 *   Limit: ulm_pair_workspace_size(ctx, capacity) must not exceed
 *   ULM_NOALLOC_SCRATCH_BYTES (about 8 M input records at 300 frames);
 *   larger `capacity` returns INVALID_ARG before anything is launched.
 *   Every call on one device shares that device's array: calls that overlap
 *   in time on one device (other streams, other contexts or threads) race and
 *   must be serialised by the caller.  The array keeps the last call's
 *   contents; the pairing overwrites every word it reads, so nothing needs
 *   clearing between calls.
 * Errors: INVALID_ARG, HIP (also if the array's address could not be looked
 * up on ctx's device).
 */
int32_t ulm_pair_planes_noalloc(ulm_ctx_t *ctx, const ulm_loc_t *locs, const int32_t *count,
                                int32_t capacity, ulm_loc3d_t *out, int32_t out_capacity,
                                int32_t *out_count, void *stream);

/* Byte offset of the stage-1 reference slices S[2][K][F][Nz][Nu] (c64) inside
 * the workspace, where rca_beamform_stage1 leaves them. */
int32_t ulm_slices_offset(const ulm_ctx_t *ctx, size_t *offset);

/* Workspace bytes for ulm_motion_estimate with lag window `max_lag`. */
int32_t ulm_motion_workspace_size(const ulm_ctx_t *ctx, int32_t max_lag, size_t *bytes);

/*
 * Rigid motion estimation on the stage-1 reference slices (Section II-A3): each
 * frame of each of the 2K slices is compared with frame `ref_frame` of the same
 * slice by the normalised cross-correlation of the two envelopes (|S|, each made
 * zero-mean; circular in the Nz x Nu grid, as an unpadded FFT correlation is);
 * the displacement is the correlation's peak within |dz|, |du| <= max_lag
 * (first maximum in raster order of (dz, du)), refined per axis by the 3-point
 * Gaussian fit of the localiser (parabolic where a value is <= 0, clamped to
 * +-0.5, none on the window edge).  The K displacements of each orientation are
 * averaged; the 3D motion takes x from the RC (x-z) slices, y from the CR (y-z)
 * slices and the mean of their axial parts.  A frame whose content moved by +d
 * pixels (frame(p) = reference(p - d)) gives +d.
 *   slices  [2][K][F][Nz][Nu] c64, device (e.g. the workspace at
 *           ulm_slices_offset after rca_beamform_stage1).
 *   disp    [2][K][F][2] f32, device: (dz, du) per slice and frame, pixels.
 *   motion  [F][3] f32, device: (dx, dy, dz) per frame, pixels.
 *   mws     workspace of at least ulm_motion_workspace_size(ctx, max_lag) bytes,
 *           256-byte aligned.
 *   max_lag 1..10, with 2 max_lag + 1 <= min(Nz, Nu).
 * Errors: INVALID_ARG, HIP.
 */
int32_t ulm_motion_estimate(ulm_ctx_t *ctx, const float *slices, int32_t ref_frame,
                            int32_t max_lag, float *disp, float *motion, void *mws,
                            size_t mws_bytes, void *stream);

/*
 * MB separation (Section II-A5): at every pixel of every filtered plane, the
 * F-point DFT over the frames, X[k] = sum_n x[n] exp(-2 pi i k n / F), an ideal
 * band-pass mask per subset and the inverse DFT.  With H = (F - 1) / 2, "up"
 * (MBs moving towards the probe, whose phase advances with this library's
 * baseband convention) keeps bins k = 1..H and "down" bins F - H..F - 1; each
 * direction is split by |k| into n_speed contiguous speed ranges, range s
 * holding |k| in [1 + floor(s H / n_speed), 1 + floor((s + 1) H / n_speed)).
 * The DC bin and, for even F, the Nyquist bin belong to no subset.
 *   filtered [2][B][F][Nz][Nu] c64, device.
 *   subsets  [2 n_speed][2][B][F][Nz][Nu] c64, device: up ranges 0..S-1 (slowest
 *            first), then down ranges 0..S-1.
 *   n_speed  1..8; F must be 2..512 with no prime factor above 7.
 * Errors: INVALID_ARG, HIP.
 */
int32_t ulm_separate(ulm_ctx_t *ctx, const float *filtered, int32_t n_speed, float *subsets,
                     void *stream);

/*
 * Learned localiser: a CNN alternative to the NCC step (the paper's outlook,
 * Section IV, names deep-learning localisation as the way past NCC on dense MB
 * populations; the network itself is this library's choice).
 *   input   I / max over the image of I, I = |filtered plane|, one channel
 *   layers  3x3 conv 1 -> 32 + ReLU, then 5 x (3x3 conv 32 -> 32 + ReLU), zero pad 1
 *   head    1x1 conv 32 -> 64 and depth-to-space by 8: heat[8z + i][8u + j] =
 *           head channel 8i + j at pixel (z, u)
 *   decode  fine pixels with heat >= threshold that are above their 3x3
 *           neighbours earlier in fine raster order and not below the later ones;
 *           position ((fine index + 1/2) / 8 - 1/2) in plane pixel units
 *   loss    mean over the fine grid of (heat - T)^2,
 *           T(q) = max over MBs of exp(-|q - (8 (x + 1/2) - 1/2)|^2 / 2)
 *           (x the MB's (z, u) in plane pixels, q a fine index, blob truncated
 *           at 4 fine pixels)
 *   update  Adam, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
 * params is a flat FP32 vector of ULM_CNN_PARAMS values:
 *   w0 [32][1][3][3], b0 [32], then for l = 1..5 wl [32][32][3][3], bl [32],
 *   then wh [64][32], bh [64]  (conv weights [out][in][dy][dx], cross-correlation).
 * Activations are BF16 (ULM_CNN_BF16) or FP32 (ULM_CNN_FP32); accumulation is
 * FP32 in both.  The CNN workspace is caller-owned device memory, 256-byte
 * aligned, of at least the size the matching *_workspace_size call returns;
 * its contents need no initialisation.
 */
#define ULM_CNN_PARAMS 48672
#define ULM_CNN_BF16 0
#define ULM_CNN_FP32 1

/* Workspace bytes for ulm_cnn_forward (train = 0) or ulm_cnn_gradients /
 * ulm_cnn_train_step (train = 1) on `batch` images of nz x nu pixels.
 * Errors: INVALID_ARG (non-positive sizes, more than 2^26 pixels, bad precision). */
int32_t ulm_cnn_workspace_size(int32_t batch, int32_t nz, int32_t nu, int32_t precision,
                               int32_t train, size_t *bytes);

/* Workspace bytes for ulm_cnn_localize on ctx's planes, `batch` images per pass
 * (includes the per-row staging of the whole ensemble's detections). */
int32_t ulm_cnn_localize_workspace_size(const ulm_ctx_t *ctx, int32_t batch, int32_t precision,
                                        size_t *bytes);

/* images [2B*F][Nz][Nu] f32, device, written: |filtered| / maximum of |filtered|
 * over the same (plane, frame) image (0 for an all-zero image).  Uses `ws`.
 * Errors: INVALID_ARG, HIP. */
int32_t ulm_cnn_images(ulm_ctx_t *ctx, const float *filtered, float *images, void *ws,
                       size_t ws_bytes, void *stream);

/* heat [batch][8 nz][8 nu] f32, device, written: the network's heatmap for
 * images [batch][nz][nu] f32 (device).  Errors: INVALID_ARG, HIP. */
int32_t ulm_cnn_forward(const float *params, const float *images, int32_t batch, int32_t nz,
                        int32_t nu, int32_t precision, float *heat, void *cnn_ws,
                        size_t cnn_ws_bytes, void *stream);

/* Loss over the batch (mean over all batch * 64 nz nu fine pixels) and its
 * gradient with respect to every parameter.
 *   mb_zu  [n_mb][2] f32, device: MB (z, u) in plane pixel units;
 *   mb_img [n_mb] i32, device: the batch image each MB belongs to (records
 *          outside [0, batch) or with |z|, |u| >= 1e6 are ignored);
 *   grad   [ULM_CNN_PARAMS] f32, device, written;  loss: f32, device, written.
 * Errors: INVALID_ARG, HIP. */
int32_t ulm_cnn_gradients(const float *params, const float *images, int32_t batch, int32_t nz,
                          int32_t nu, const float *mb_zu, const int32_t *mb_img, int32_t n_mb,
                          int32_t precision, float *grad, float *loss, void *cnn_ws,
                          size_t cnn_ws_bytes, void *stream);

/* ulm_cnn_gradients into the workspace, then one Adam update of params with the
 * moment buffers adam_m, adam_v ([ULM_CNN_PARAMS] f32, device, zero before the
 * first step); `step` counts updates from 1 (bias correction).
 * Errors: INVALID_ARG, HIP. */
int32_t ulm_cnn_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr,
                           const float *images, int32_t batch, int32_t nz, int32_t nu,
                           const float *mb_zu, const int32_t *mb_img, int32_t n_mb,
                           int32_t precision, float *loss, void *cnn_ws, size_t cnn_ws_bytes,
                           void *stream);

/* CNN localisation of every filtered plane, `batch` images per pass.  Output as
 * ncc_localize: records sorted by (plane, frame, iz, iu) and then by the fine
 * position inside the pixel; `ncc` holds the heat value and `intensity` the
 * envelope |filtered| at (iz, iu).  A plane row with more than max(16, Nu/2)
 * peaks keeps the first ones and flags ULM_ERR_OVERFLOW in ulm_check_status.
 * Errors: INVALID_ARG, HIP. */
int32_t ulm_cnn_localize(ulm_ctx_t *ctx, const float *params, const float *filtered,
                         float threshold, int32_t batch, int32_t precision, ulm_loc_t *locs,
                         int32_t capacity, int32_t *count, void *ws, size_t ws_bytes,
                         void *cnn_ws, size_t cnn_ws_bytes, void *stream);

/* The whole path with the learned localiser in place of NCC:
 * rca_beamform_proj -> svd_clutter_filter -> ulm_cnn_localize.  Arguments as
 * ulm_reconstruct_ensemble, plus the network's `params`, `threshold`, `batch`,
 * `precision` and its workspace `cnn_ws` as ulm_cnn_localize; the CNN's
 * arguments are checked before any work is queued.  Errors: INVALID_ARG, HIP. */
int32_t ulm_reconstruct_ensemble_cnn(ulm_ctx_t *ctx, const float *iq, float *proj,
                                     double *eigvals, const float *params, float threshold,
                                     int32_t batch, int32_t precision, ulm_loc_t *locs,
                                     int32_t capacity, int32_t *count, void *ws, size_t ws_bytes,
                                     void *cnn_ws, size_t cnn_ws_bytes, ulm_timing_t *timing,
                                     void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ULMPROJ_H */
