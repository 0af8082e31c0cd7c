/*
 * Oracle (test infrastructure only): FP64 delay-and-sum loops for row-column
 * plane-wave imaging.  Plain, unblocked loops that follow the definitions of
 * the paper's Section II-A1 (two-stage beamforming: a stage-1 reference slice
 * per transmit) and the conventional full-3D DAS it approximates.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  It shares no code with the HIP path.
 *
 * Geometry (a reading of the paper, which does not state it):
 *   element e of the receive array at  p_e = (e - (N-1)/2) * pitch
 *   transmit delay of a plane wave steered by theta, evaluated at (v, z):
 *       tau_tx = (z cos(theta) + v sin(theta) + (L/2)|sin(theta)|) / c,
 *       L = (N-1) * pitch  (firing delays are non-negative)
 *   receive delay of line element e at lateral position u, depth z:
 *       tau_rx = sqrt((u - p_e)^2 + z^2) / c
 *   IQ sample index s = (tau - t_start) * fs, linear interpolation between
 *   floor(s) and floor(s)+1; samples outside [0, Ns-1] are zero.
 *   beamformed value: IQ(s) * exp(+i 2 pi f0 (tau - 2 z / c))
 *   (baseband with respect to the nominal round trip 2z/c).
 *
 * Complex arrays are interleaved (re, im) doubles.
 */
#include <math.h>
#include <stddef.h>

typedef struct {
    int n_elem;
    double pitch, c, f0, fs, t_start;
    int n_samp;
} oracle_probe_t;

static void iq_lerp(const double *ch, int ns, double s, double *re, double *im)
{
    double fl = floor(s);
    long i0 = (long)fl;
    double fr = s - fl;
    double a_re = 0.0, a_im = 0.0, b_re = 0.0, b_im = 0.0;
    if (i0 >= 0 && i0 < ns) { a_re = ch[2 * i0]; a_im = ch[2 * i0 + 1]; }
    if (i0 + 1 >= 0 && i0 + 1 < ns) { b_re = ch[2 * (i0 + 1)]; b_im = ch[2 * (i0 + 1) + 1]; }
    *re = (1.0 - fr) * a_re + fr * b_re;
    *im = (1.0 - fr) * a_im + fr * b_im;
}

/* One voxel of DAS for transmit angle theta at (u, v, z), summed over all
 * receive channels of one (frame, orientation, angle) channel block. */
static void das_point(const double *blk, const oracle_probe_t *pr, double theta,
                      double u, double v, double z, double *out_re, double *out_im)
{
    const double PI = 3.14159265358979323846;
    double L = (pr->n_elem - 1) * pr->pitch;
    double tau_tx = (z * cos(theta) + v * sin(theta) + 0.5 * L * fabs(sin(theta))) / pr->c;
    double acc_re = 0.0, acc_im = 0.0;
    for (int e = 0; e < pr->n_elem; ++e) {
        double pe = (e - 0.5 * (pr->n_elem - 1)) * pr->pitch;
        double tau = tau_tx + sqrt((u - pe) * (u - pe) + z * z) / pr->c;
        double s = (tau - pr->t_start) * pr->fs;
        double x_re, x_im;
        iq_lerp(blk + (size_t)e * pr->n_samp * 2, pr->n_samp, s, &x_re, &x_im);
        double ph = 2.0 * PI * pr->f0 * (tau - 2.0 * z / pr->c);
        double c_ = cos(ph), s_ = sin(ph);
        acc_re += x_re * c_ - x_im * s_;
        acc_im += x_re * s_ + x_im * c_;
    }
    *out_re = acc_re;
    *out_im = acc_im;
}

/*
 * Stage 1: for every frame f, orientation o and transmit k, the reference
 * slice S[o][k][f][z][u] at v = v_ref.
 * iq:  [F][O][K][Nc][Ns] complex;  out: [O][K][F][Nz][Nu] complex.
 */
void oracle_das_stage1(const double *iq, int F, int O, int K, const double *angles,
                       const oracle_probe_t *pr, int nu, int nz, double u0, double du,
                       double z0, double dz, double v_ref, double *out)
{
    size_t blk_len = (size_t)pr->n_elem * pr->n_samp * 2;
    long rows = (long)O * K * F * nz;
#pragma omp parallel for schedule(dynamic, 4)
    for (long r = 0; r < rows; ++r) {
        int l = (int)(r % nz);
        int f = (int)((r / nz) % F);
        int k = (int)((r / ((long)nz * F)) % K);
        int o = (int)(r / ((long)nz * F * K));
        const double *blk = iq + (((size_t)f * O + o) * K + k) * blk_len;
        double z = z0 + l * dz;
        double *dst = out + ((((size_t)o * K + k) * F + f) * nz + l) * (size_t)nu * 2;
        for (int i = 0; i < nu; ++i) {
            double u = u0 + i * du;
            das_point(blk, pr, angles[k], u, v_ref, z, &dst[2 * i], &dst[2 * i + 1]);
        }
    }
}

/*
 * Conventional full-3D DAS of every voxel (u, v_m, z) for v indices
 * m in [m_lo, m_hi), summed over those slices (a sum projection of the
 * beamformed volume along v).  One transmit angle per output block.
 * out: [O][K][F][Nz][Nu] complex.
 */
void oracle_das_3d_slab(const double *iq, int F, int O, int K, const double *angles,
                        const oracle_probe_t *pr, int nu, int nz, double u0, double du,
                        double z0, double dz, double v0, double dv, int m_lo, int m_hi,
                        double *out)
{
    size_t blk_len = (size_t)pr->n_elem * pr->n_samp * 2;
    long rows = (long)O * K * F * nz;
#pragma omp parallel for schedule(dynamic, 2)
    for (long r = 0; r < rows; ++r) {
        int l = (int)(r % nz);
        int f = (int)((r / nz) % F);
        int k = (int)((r / ((long)nz * F)) % K);
        int o = (int)(r / ((long)nz * F * K));
        const double *blk = iq + (((size_t)f * O + o) * K + k) * blk_len;
        double z = z0 + l * dz;
        double *dst = out + ((((size_t)o * K + k) * F + f) * nz + l) * (size_t)nu * 2;
        for (int i = 0; i < nu; ++i) {
            double u = u0 + i * du;
            double sre = 0.0, sim = 0.0;
            for (int m = m_lo; m < m_hi; ++m) {
                double re, im;
                das_point(blk, pr, angles[k], u, v0 + m * dv, z, &re, &im);
                sre += re;
                sim += im;
            }
            dst[2 * i] = sre;
            dst[2 * i + 1] = sim;
        }
    }
}
