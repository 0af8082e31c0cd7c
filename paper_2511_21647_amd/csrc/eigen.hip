// FP64 Hermitian eigensolver for the clutter filter (paper Section II-A2: the
// covariance of the Casorati matrix is eigendecomposed and the eigenvectors of
// the largest eigenvalues span the clutter subspace).
//
// eigen_coop_kernel: W work-groups per plane, all on one XCD (the plane's
// grid slots are dealt to a single XCD), launched cooperatively.
//   1. Householder reduction to real tridiagonal form T = Q^H C Q (the
//      unblocked Hermitian reduction).  Column j of C lives in the LDS of
//      work-group j mod W for the whole reduction.  The rank-2 update of step
//      k-1 is fused with the matrix-vector product of step k, so each step
//      costs two grid barriers: one after the owner of column k publishes the
//      reflector v_k, one after every work-group publishes its part of
//      p_k = tau_k A v_k.
//   2. Every eigenvalue of T by bisection on Sturm counts (spread over the
//      plane's work-groups).
//   3. Work-group 0: inverse iteration (partial-pivoting tridiagonal LU) for
//      the c largest eigenvalues, two Gram-Schmidt passes, and the
//      back-transformation x = H_0 H_1 ... H_{F-2} y.
// Grid barriers spin on an agent-scope counter with a bounded wait: a work-
// group that waits too long flags the status word and exits, so every wave
// always finishes.
#include "common.h"

#include <float.h>

namespace ulm {

constexpr int kCoopThreads = 256;
constexpr int kCoopWaves = kCoopThreads / 64;

struct EigArgs {
    const double2 *C;   // [planes][F][F] covariance (full Hermitian)
    double2 *H;         // [planes][F][F] row k: Householder vector v_k (entries k+1..F-1)
    double2 *tau;       // [planes][F]
    double *d, *e;      // [planes][F]
    double *lam;        // [planes][F] eigenvalues, descending
    double *lam_out;    // optional copy of lam
    double2 *V;         // [planes][F][c] clutter eigenvectors
    double *tscr;       // [planes][c][6][F]
    double2 *xscr;      // [planes][c][F]
    double2 *vbuf;      // [planes][F] reflector of the current step
    double2 *pbuf;      // [planes][F]
    double *dots;       // [planes][W][2]
    double *scal;       // unused
    int *bar;           // [planes] barrier counters, zero at launch
    int *flag;          // [planes] non-finite input
    int *status;
    int F, c, W, planes;
};

__device__ inline double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cjmul2(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double bsum(double v, double *red) {
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kCoopWaves; ++i) s += red[i];
    return s;
}
__device__ inline double bmax(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < kCoopWaves; ++i) s = fmax(s, red[i]);
    return s;
}

// Cross-work-group traffic uses relaxed agent-scope atomics: plain loads and
// stores with the system-coherence bit, so no L2 write-back or invalidation is
// needed inside the reduction.  A work-group arrives at a barrier only after its
// own stores have completed (s_waitcnt 0).
__device__ inline void st_c(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_c(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_c2(double2 *p, double2 v) {
    st_c((double *)p, v.x);
    st_c((double *)p + 1, v.y);
}
__device__ inline double2 ld_c2(const double2 *p) {
    return make_double2(ld_c((const double *)p), ld_c((const double *)p + 1));
}

// Grid barrier among the W work-groups of one plane.  Returns false if the
// wait timed out (the caller then exits).
__device__ inline bool plane_barrier(int *cnt, int target, int *abort_s, int *status) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1 << 23)) {
                *abort_s = 1;
                atomicOr(status, kStatusBarrier);
                break;
            }
        }
    }
    __syncthreads();
    return *abort_s == 0;
}

__device__ inline int sturm(const double *d, const double *e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
        if (fabs(q) <= pivmin) q = -pivmin;
        q = d[i] - x - e2[i - 1] / q;
        cnt += q < 0.0;
    }
    return cnt;
}

// Reflector of the unblocked Hermitian reduction (LAPACK's elementary
// reflector convention): H^H x = (beta, 0, ...)^T, H = I - tau v v^H, v_0 = 1.
// x = col[k+1 .. F); computed identically by every work-group.
__device__ inline void reflector(const double2 *col, int k, int F, double *red, double2 *v,
                                 double2 &tk, double &beta) {
    double nrm = 0.0;
    for (int i = k + 2 + threadIdx.x; i < F; i += kCoopThreads)
        nrm += col[i].x * col[i].x + col[i].y * col[i].y;
    nrm = bsum(nrm, red);
    const double2 alpha = col[k + 1];
    tk = make_double2(0.0, 0.0);
    beta = alpha.x;
    double2 scale = make_double2(0.0, 0.0);
    if (nrm > 0.0 || alpha.y != 0.0) {
        beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + nrm), alpha.x);
        tk = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double2 den = make_double2(alpha.x - beta, alpha.y);
        const double dd = den.x * den.x + den.y * den.y;
        scale = make_double2(den.x / dd, -den.y / dd);
    }
    for (int i = k + 1 + threadIdx.x; i < F; i += kCoopThreads)
        v[i] = (i == k + 1) ? make_double2(1.0, 0.0) : cmul2(col[i], scale);
}

// Pending rank-2 update A -= v p^H + p v^H + a2r v v^H applied to column j.
__device__ inline double2 pending(double2 x, double2 vi, double2 pi, double2 cpj, double2 cvj,
                                  double a2r) {
    const double2 u1 = cmul2(vi, cpj), u2 = cmul2(pi, cvj), u3 = cmul2(vi, cvj);
    return make_double2(x.x - (u1.x + u2.x + a2r * u3.x), x.y - (u1.y + u2.y + a2r * u3.y));
}

__global__ __launch_bounds__(kCoopThreads) void eigen_coop_kernel(EigArgs a)
{
    const int g = blockIdx.x, xcd = g & 7, slot = g >> 3;
    const int W = a.W, F = a.F, c = a.c;
    const int plane = xcd + 8 * (slot / W), w = slot % W;
    if (plane >= a.planes) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int ncol = cdiv(F, W);

    extern __shared__ double2 lds2[];
    double2 *Acol = lds2;                     // [ncol][F]: local column q = global column w + q W
    double2 *sv = Acol + (size_t)ncol * F;    // v of the pending update
    double2 *sp = sv + F;                     // p of the pending update
    double2 *svn = sp + F;                    // v of the current step
    double2 *scol = svn + F;                  // column k as published by its owner
    __shared__ double red[kCoopWaves];
    __shared__ double2 wpart[kCoopWaves];
    __shared__ int abort_s;
    if (t == 0) abort_s = 0;

    const double2 *C = a.C + (size_t)plane * F * F;
    double2 *H = a.H + (size_t)plane * F * F;
    double2 *tau = a.tau + (size_t)plane * F;
    double *d = a.d + (size_t)plane * F, *e = a.e + (size_t)plane * F;
    // double-buffered exchange areas (by step parity): p, the next column, dots
    double2 *pbuf = a.pbuf + (size_t)plane * 2 * F;
    double2 *cbuf = a.vbuf + (size_t)plane * 2 * F;
    double *dots = a.dots + (size_t)plane * 2 * 64;
    int *cnt = a.bar + plane;
    int nbar = 0;

    // load own columns (A[i][j] = conj(C[j][i]), contiguous in i) and check them
    double bad = 0.0;
    for (int q = 0; q < ncol; ++q) {
        const int j = w + q * W;
        if (j >= F) break;
        for (int i = t; i < F; i += kCoopThreads) {
            const double2 v = C[(size_t)j * F + i];
            if (!isfinite(v.x) || !isfinite(v.y)) bad = 1.0;
            Acol[(size_t)q * F + i] = make_double2(v.x, -v.y);
        }
    }
    for (int i = t; i < F; i += kCoopThreads) {
        sv[i] = sp[i] = make_double2(0.0, 0.0);
        scol[i] = make_double2(0.0, 0.0);
    }
    bad = bmax(bad, red);
    if (t == 0 && bad > 0.0) atomicOr(a.flag + plane, 1);
    // the owner of column 0 publishes it
    if (w == 0)
        for (int i = t; i < F; i += kCoopThreads) st_c2(cbuf + i, Acol[i]);
    if (!plane_barrier(cnt, ++nbar * W, &abort_s, a.status)) return;
    if (__hip_atomic_load(a.flag + plane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        if (w == 0) {
            double2 *V = a.V + (size_t)plane * F * (c > 0 ? c : 1);
            for (int i = t; i < F * c; i += kCoopThreads) V[i] = make_double2(0.0, 0.0);
            for (int i = t; i < F; i += kCoopThreads) {
                a.lam[(size_t)plane * F + i] = __builtin_nan("");
                if (a.lam_out) a.lam_out[(size_t)plane * F + i] = __builtin_nan("");
            }
            if (t == 0) atomicOr(a.status, kStatusNumeric);
        }
        return;
    }
    for (int i = t; i < F; i += kCoopThreads) scol[i] = ld_c2(cbuf + i);
    __syncthreads();

    double a2r = 0.0;   // 2 Re(alpha) of the pending rank-2 update (step k-1)
    for (int k = 0; k + 1 < F; ++k) {
        const int par = k & 1;
        // column k: pending update of step k-1 (rows >= k), then the reflector
        if (k > 0) {
            const double2 cpk = make_double2(sp[k].x, -sp[k].y), cvk = make_double2(sv[k].x, -sv[k].y);
            for (int i = k + t; i < F; i += kCoopThreads) scol[i] = pending(scol[i], sv[i], sp[i], cpk, cvk, a2r);
            __syncthreads();
        }
        double2 tk;
        double beta;
        reflector(scol, k, F, red, svn, tk, beta);
        __syncthreads();
        if (w == k % W) {
            for (int i = k + 1 + t; i < F; i += kCoopThreads) st_c2(H + (size_t)k * F + i, svn[i]);
            if (t == 0) {
                st_c(d + k, scol[k].x);
                st_c(e + k, beta);
                st_c2(tau + k, tk);
            }
        }
        // own columns j > k: pending update, then p_j = tau_k sum_i conj(A[i][j]) v_i
        double2 part = make_double2(0.0, 0.0);
        for (int q = wave; q < ncol; q += kCoopWaves) {
            const int j = w + q * W;
            if (j <= k || j >= F) continue;
            double2 *col = Acol + (size_t)q * F;
            const double2 cpj = make_double2(sp[j].x, -sp[j].y), cvj = make_double2(sv[j].x, -sv[j].y);
            double ar = 0.0, ai = 0.0;
            for (int i = k + 1 + lane; i < F; i += 64) {
                double2 x = col[i];
                if (k > 0) {
                    x = pending(x, sv[i], sp[i], cpj, cvj, a2r);
                    col[i] = x;
                }
                const double2 pr = cjmul2(x, svn[i]);
                ar += pr.x;
                ai += pr.y;
            }
            ar = wsum(ar);
            ai = wsum(ai);
            const double2 pj = cmul2(tk, make_double2(ar, ai));
            if (lane == 0) st_c2(pbuf + par * F + j, pj);
            const double2 pv = cjmul2(pj, svn[j]);
            part.x += pv.x;
            part.y += pv.y;
            if (j == k + 1)    // publish the next column (rows > k) for every work-group
                for (int i = k + 1 + lane; i < F; i += 64) st_c2(cbuf + par * F + i, col[i]);
        }
        if (lane == 0) wpart[wave] = part;
        __syncthreads();
        if (t == 0) {
            double2 s = make_double2(0.0, 0.0);
            for (int q = 0; q < kCoopWaves; ++q) { s.x += wpart[q].x; s.y += wpart[q].y; }
            st_c(dots + par * 64 + 2 * w, s.x);
            st_c(dots + par * 64 + 2 * w + 1, s.y);
        }
        if (!plane_barrier(cnt, ++nbar * W, &abort_s, a.status)) return;
        double pr = 0.0, pi = 0.0;
        for (int q = 0; q < W; ++q) {
            pr += ld_c(dots + par * 64 + 2 * q);
            pi += ld_c(dots + par * 64 + 2 * q + 1);
        }
        // alpha = -1/2 tau (p^H v); the pending update uses 2 Re(alpha)
        const double2 al = cmul2(make_double2(-0.5 * tk.x, -0.5 * tk.y), make_double2(pr, pi));
        a2r = 2.0 * al.x;
        for (int i = t; i < F; i += kCoopThreads) {
            if (i > k) {
                sp[i] = ld_c2(pbuf + par * F + i);
                sv[i] = svn[i];
                scol[i] = ld_c2(cbuf + par * F + i);
            } else {
                sp[i] = sv[i] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
    }
    // last diagonal entry: pending update of step F-2 applied to A[F-1][F-1]
    if (w == 0 && t == 0) {
        double dl = scol[F - 1].x;
        if (F >= 2) {
            const double2 vi = sv[F - 1], pi = sp[F - 1];
            dl -= 2.0 * (vi.x * pi.x + vi.y * pi.y) + a2r * (vi.x * vi.x + vi.y * vi.y);
        }
        st_c(d + F - 1, dl);
        st_c(e + F - 1, 0.0);
        st_c2(tau + F - 1, make_double2(0.0, 0.0));
    }
    if (!plane_barrier(cnt, ++nbar * W, &abort_s, a.status)) return;

    // 2. eigenvalues by bisection, spread over the plane's work-groups
    double *sd = (double *)lds2;
    double *se2 = sd + F;
    double lo_b = 1e300, hi_b = -1e300, emax = 0.0;
    for (int i = t; i < F; i += kCoopThreads) {
        const double di = ld_c(d + i), ei = (i + 1 < F) ? ld_c(e + i) : 0.0;
        const double em = (i > 0) ? ld_c(e + i - 1) : 0.0;
        const double r = fabs(em) + fabs(ei);
        lo_b = fmin(lo_b, di - r);
        hi_b = fmax(hi_b, di + r);
        sd[i] = di;
        se2[i] = ei * ei;
        emax = fmax(emax, ei * ei);
    }
    hi_b = bmax(hi_b, red);
    lo_b = -bmax(-lo_b, red);
    emax = bmax(emax, red);
    const double tnorm = fmax(fabs(lo_b), fabs(hi_b));
    const double pivmin = fmax(DBL_MIN, DBL_MIN * emax);
    lo_b -= 2.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
    hi_b += 2.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
    double *lam = a.lam + (size_t)plane * F;
    for (int idx = w * kCoopThreads + t; idx < F; idx += W * kCoopThreads) {
        const int target = F - 1 - idx;
        double lo = lo_b, hi = hi_b;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi || hi - lo <= 2.0 * DBL_EPSILON * tnorm) break;
            if (sturm(sd, se2, F, mid, pivmin) > target) hi = mid; else lo = mid;
        }
        st_c(lam + idx, 0.5 * (lo + hi));
        if (a.lam_out) a.lam_out[(size_t)plane * F + idx] = 0.5 * (lo + hi);
    }
    if (!plane_barrier(cnt, ++nbar * W, &abort_s, a.status)) return;
    if (w != 0 || c <= 0) return;
    // everything the other work-groups wrote is read through L2 from here on
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    // 3. inverse iteration for the c largest eigenvalues (one thread each)
    double *ts = a.tscr + (size_t)plane * c * 6 * F;
    if (t < c) {
        double *u0 = ts + (size_t)t * 6 * F;
        double *u1 = u0 + F, *u2 = u1 + F, *ml = u2 + F, *b = ml + F, *swp = b + F;
        const double lm = lam[t];
        const double tiny = DBL_EPSILON * tnorm + pivmin;
        for (int i = 0; i < F; ++i) {
            u0[i] = sd[i] - lm;
            u1[i] = (i + 1 < F) ? e[i] : 0.0;
            u2[i] = 0.0;
            swp[i] = 0.0;
        }
        for (int i = 0; i + 1 < F; ++i) {
            const double sub = e[i];
            if (fabs(u0[i]) >= fabs(sub)) {
                if (u0[i] == 0.0) u0[i] = tiny;
                ml[i] = sub / u0[i];
                u0[i + 1] -= ml[i] * u1[i];
            } else {
                const double l = u0[i] / sub;
                const double t1 = u0[i + 1];
                const double t2 = (i + 2 < F) ? u1[i + 1] : 0.0;
                u0[i] = sub;
                u0[i + 1] = u1[i] - l * t1;
                if (i + 2 < F) u1[i + 1] = -l * t2;
                u1[i] = t1;
                u2[i] = t2;
                ml[i] = l;
                swp[i] = 1.0;
            }
        }
        if (u0[F - 1] == 0.0) u0[F - 1] = tiny;
        for (int i = 0; i < F; ++i) b[i] = 1.0 + 0.37 * sin(0.731 * i + 1.3 * t);
        for (int it = 0; it < 3; ++it) {
            for (int i = 0; i + 1 < F; ++i) {
                if (swp[i] != 0.0) { const double x = b[i]; b[i] = b[i + 1]; b[i + 1] = x; }
                b[i + 1] -= ml[i] * b[i];
            }
            b[F - 1] /= u0[F - 1];
            if (F >= 2) b[F - 2] = (b[F - 2] - u1[F - 2] * b[F - 1]) / u0[F - 2];
            for (int i = F - 3; i >= 0; --i) b[i] = (b[i] - u1[i] * b[i + 1] - u2[i] * b[i + 2]) / u0[i];
            double n2 = 0.0;
            for (int i = 0; i < F; ++i) n2 += b[i] * b[i];
            const double inv = 1.0 / sqrt(n2);
            for (int i = 0; i < F; ++i) b[i] *= inv;
        }
    }
    __syncthreads();
    // two passes of classical Gram-Schmidt: vector i against all earlier ones at
    // once (wave-level dots), then normalise
    double *gdot = (double *)(lds2) + 2 * F;       // [c] after sd, se2
    for (int i = 0; i < c; ++i) {
        double *bi = ts + (size_t)i * 6 * F + 4 * F;
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = wave; j < i; j += kCoopWaves) {
                const double *bj = ts + (size_t)j * 6 * F + 4 * F;
                double s = 0.0;
                for (int q = lane; q < F; q += 64) s += bj[q] * bi[q];
                s = wsum(s);
                if (lane == 0) gdot[j] = s;
            }
            __syncthreads();
            for (int q = t; q < F; q += kCoopThreads) {
                double x = bi[q];
                for (int j = 0; j < i; ++j) x -= gdot[j] * ts[(size_t)j * 6 * F + 4 * F + q];
                bi[q] = x;
            }
            __syncthreads();
        }
        double n2 = 0.0;
        for (int q = t; q < F; q += kCoopThreads) n2 += bi[q] * bi[q];
        n2 = bsum(n2, red);
        const double inv = 1.0 / sqrt(n2);
        for (int q = t; q < F; q += kCoopThreads) bi[q] *= inv;
        __syncthreads();
    }
    // back-transformation x = H_0 H_1 ... H_{F-2} y, one wave per vector
    double2 *xs = a.xscr + (size_t)plane * c * F;
    for (int i = t; i < c * F; i += kCoopThreads)
        xs[i] = make_double2(ts[(size_t)(i / F) * 6 * F + 4 * F + (i % F)], 0.0);
    __syncthreads();
    for (int vi = wave; vi < c; vi += kCoopWaves) {
        double2 *x = xs + (size_t)vi * F;
        for (int k = F - 2; k >= 0; --k) {
            const double2 tk = tau[k];
            if (tk.x == 0.0 && tk.y == 0.0) continue;
            const double2 *v = H + (size_t)k * F;
            double sr = 0.0, si = 0.0;
            for (int q = k + 1 + lane; q < F; q += 64) {
                const double2 p = cjmul2(v[q], x[q]);
                sr += p.x;
                si += p.y;
            }
            sr = wsum(sr);
            si = wsum(si);
            const double2 s = cmul2(tk, make_double2(sr, si));
            for (int q = k + 1 + lane; q < F; q += 64) {
                const double2 p = cmul2(v[q], s);
                x[q] = make_double2(x[q].x - p.x, x[q].y - p.y);
            }
        }
    }
    __syncthreads();
    double2 *V = a.V + (size_t)plane * F * c;
    for (int i = t; i < c * F; i += kCoopThreads) {
        const int vi = i % c, f = i / c;
        V[(size_t)f * c + vi] = xs[(size_t)vi * F + f];
    }
}

int eigen_coop_width(int F) { return std::max(1, std::min(32, cdiv(F, 10))); }

size_t eigen_coop_lds(int F) {
    const int W = eigen_coop_width(F);
    // own columns + 4 vectors; the tail reuses it for d, e^2 and c dots
    return ((size_t)cdiv(F, W) * F + 4 * (size_t)F) * sizeof(double2) + 64 * sizeof(double);
}

hipError_t launch_eigen_coop(const EigArgs &args, hipStream_t st) {
    const int slots = cdiv(args.planes, 8) * args.W;
    dim3 grid(8 * slots), block(kCoopThreads);
    EigArgs a = args;
    void *params[] = {&a};
    return hipLaunchCooperativeKernel((const void *)eigen_coop_kernel, grid, block, params,
                                      (unsigned)eigen_coop_lds(args.F), st);
}

}  // namespace ulm
