// Forward model of RCA plane-wave IQ channel data (input generator; it is not
// part of the timed path).  A linear Gaussian-pulse model of the acquisition
// of the paper's Section II-C: every scatterer adds
//   amp * exp(-(t_s - tau)^2 / (2 sigma_t^2)) * exp(-i 2 pi f0 tau)
// to each element's samples, tau = plane-wave transmit delay + element receive
// delay.  Channel noise: Philox4x32-10 (Salmon et al., SC 2011) keyed by the
// seed and the sample's flat index, Box-Muller to a complex Gaussian.
//
// One work-group per (frame, orientation, angle, group of 8 elements); the
// group's sample vectors accumulate in LDS.
#include "common.h"

#include <math.h>

namespace ulm {

constexpr int kSimGroup = 8;

struct SimParams {
    double c, f0, fs, t_start, pitch, half_l;
    double inv_2sig2_samples;   // 1 / (2 sigma_t^2 fs^2)
    int reach;                  // samples either side of the pulse centre
    double noise_scale;         // noise_sigma / sqrt(2)
    unsigned long long seed;
};

__device__ inline void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * ctr[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t c1 = ctr[1], c3 = ctr[3];
        ctr[0] = hi1 ^ c1 ^ k0;
        ctr[1] = lo1;
        ctr[2] = hi0 ^ c3 ^ k1;
        ctr[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ __launch_bounds__(256) void sim_kernel(const double *__restrict__ pos,
                                                  const double2 *__restrict__ amp, int n_scat,
                                                  const double *__restrict__ angles,
                                                  float2 *__restrict__ iq, SimParams sp, int K,
                                                  int Nc, int Ns)
{
    extern __shared__ float sacc[];                 // [kSimGroup][Ns] re, then im
    float *are = sacc, *aim = sacc + kSimGroup * Ns;
    const int jg = blockIdx.x, ok = blockIdx.y, f = blockIdx.z;
    const int o = ok / K, k = ok % K;
    for (int e = threadIdx.x; e < 2 * kSimGroup * Ns; e += blockDim.x) sacc[e] = 0.f;
    __syncthreads();

    const double th = angles[k];
    const double sth = sin(th), cth = cos(th), ast = fabs(sth);
    const double half_ap = 0.5 * (Nc - 1);
    const double *pf = pos + (size_t)f * n_scat * 3;
    for (int q = threadIdx.x; q < n_scat; q += blockDim.x) {
        const double x = pf[3 * q], y = pf[3 * q + 1], z = pf[3 * q + 2];
        const double u = o == 0 ? x : y, v = o == 0 ? y : x;
        const double ttx = (z * cth + v * sth + sp.half_l * ast) / sp.c;
        const double2 a = amp[q];
        for (int jj = 0; jj < kSimGroup; ++jj) {
            const int j = jg * kSimGroup + jj;
            if (j >= Nc) break;
            const double ej = (j - half_ap) * sp.pitch;
            const double tau = ttx + sqrt((u - ej) * (u - ej) + z * z) / sp.c;
            const double sc = (tau - sp.t_start) * sp.fs;
            const double cyc = sp.f0 * tau;
            const float fr = (float)(cyc - rint(cyc));
            float sn, cs;
            sincospif(2.0f * fr, &sn, &cs);           // exp(-i 2 pi f0 tau) = cs - i sn
            const float cr = (float)a.x * cs + (float)a.y * sn;
            const float ci = (float)a.y * cs - (float)a.x * sn;
            const int s_lo = max(0, (int)ceil(sc - sp.reach));
            const int s_hi = min(Ns - 1, (int)floor(sc + sp.reach));
            const float g = (float)sp.inv_2sig2_samples;
            for (int s = s_lo; s <= s_hi; ++s) {
                const float dt = (float)((double)s - sc);
                const float w = __expf(-dt * dt * g);
                atomicAdd(&are[jj * Ns + s], w * cr);
                atomicAdd(&aim[jj * Ns + s], w * ci);
            }
        }
    }
    __syncthreads();
    const size_t base = (((size_t)f * 2 + o) * K + k) * Nc;
    const uint32_t k0 = (uint32_t)sp.seed, k1 = (uint32_t)(sp.seed >> 32);
    for (int e = threadIdx.x; e < kSimGroup * Ns; e += blockDim.x) {
        const int jj = e / Ns, s = e % Ns;
        const int j = jg * kSimGroup + jj;
        if (j >= Nc) continue;
        const size_t n = (base + j) * Ns + s;
        float2 v = make_float2(are[e], aim[e]);
        if (sp.noise_scale > 0.0) {
            uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), 0u, 0u};
            philox4x32_10(ctr, k0, k1);
            const double u1 = ((double)ctr[0] + 1.0) * (1.0 / 4294967296.0);
            const double u2 = (double)ctr[1] * (1.0 / 4294967296.0);
            const double r = sqrt(-2.0 * log(u1)) * sp.noise_scale;
            double sn, cs;
            sincospi(2.0 * u2, &sn, &cs);
            v.x += (float)(r * cs);
            v.y += (float)(r * sn);
        }
        iq[n] = v;
    }
}

hipError_t launch_sim(const ulm_ctx *ctx, const double *pos, const double *amp, int n_scat,
                      uint64_t seed, double noise_sigma, float *iq, const double *angles_dev,
                      hipStream_t st)
{
    const ulm_config_t &c = ctx->cfg;
    SimParams sp;
    sp.c = c.c;
    sp.f0 = c.f0;
    sp.fs = c.fs;
    sp.t_start = c.t_start;
    sp.pitch = c.pitch;
    sp.half_l = 0.5 * (c.n_elem - 1) * c.pitch;
    const double sig = sqrt(2.0 * log(2.0)) / (M_PI * c.bandwidth * c.f0);
    const double sig_s = sig * c.fs;
    sp.inv_2sig2_samples = 1.0 / (2.0 * sig_s * sig_s);
    sp.reach = (int)ceil(sqrt(2.0 * log(1e9)) * sig_s);
    sp.noise_scale = noise_sigma / sqrt(2.0);
    sp.seed = seed;
    const int Ns = c.n_samp;
    const size_t lds = (size_t)2 * kSimGroup * Ns * sizeof(float);
    dim3 grid(cdiv(c.n_elem, kSimGroup), 2 * c.n_angles, c.n_frames);
    hipLaunchKernelGGL(sim_kernel, grid, dim3(256), lds, st, pos, (const double2 *)amp, n_scat,
                       angles_dev, (float2 *)iq, sp, c.n_angles, c.n_elem, Ns);
    return hipGetLastError();
}


}  // namespace ulm
