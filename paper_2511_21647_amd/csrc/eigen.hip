// FP64 Hermitian eigensolver for the clutter filter (paper Section II-A2: the
// covariance of the Casorati matrix is eigendecomposed and the eigenvectors of
// the largest eigenvalues span the clutter subspace).
//
// eigen_coop_kernel: W work-groups per plane, launched cooperatively; the
// plane's grid slots are dealt to one XCD (see the exchange modes below).
//   1. Householder reduction to real tridiagonal form T = Q^H C Q (the
//      unblocked Hermitian reduction).  Column j of C lives in the LDS of
//      work-group j mod W for the whole reduction.  The rank-2 update of step
//      k-1 is applied lazily, fused with the matrix-vector product of step k,
//      and every work-group forms the reflector v_k itself from the published
//      column k, so each step costs one grid barrier: after every work-group
//      has published its part of p_k = tau_k A v_k and the owner of column k+1
//      has published that column; every work-group then reads all of p, forms
//      p^H v itself and applies the step's update to column k+1.
//   2. Every eigenvalue of T by multisection on Sturm counts (16 lanes per
//      eigenvalue, 16 points per round), spread over the plane's work-groups.
//   3. Inverse iteration (partial-pivoting tridiagonal LU in LDS) for the c
//      largest eigenvalues, one eigenvector per work-group.
//   4. Work-group 0: two Gram-Schmidt passes over the c vectors in LDS.
//   5. Back-transformation x = H_0 H_1 ... H_{F-2} y, one work-group per
//      vector with x in registers.
// Grid barriers spin on per-work-group flags with a bounded wait: a work-group
// that waits too long flags the status word and exits, so every wave always
// finishes.
#include "eigen.h"

#include <float.h>

namespace ulm {

constexpr int kCoopThreads = 256;
constexpr int kCoopWaves = kCoopThreads / 64;
constexpr int kCoopRows = 8;     // rows per lane of a 64-lane column: F <= 512
constexpr int kPoints = 16;      // multisection points per eigenvalue and round
constexpr int kGroups = 64 / kPoints;   // eigenvalues per wave: F <= kGroups x 4 waves x W


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
__device__ inline double2 bsum2(double a, double b, double2 *red) {
    a = wsum(a);
    b = wsum(b);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(a, b);
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < kCoopWaves; ++i) {
        s.x += red[i].x;
        s.y += red[i].y;
    }
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

// Cross-work-group traffic.  A plane's work-groups are dealt to one XCD when
// the kernel runs alone; kernels running at the same time on other streams
// shift the dispatcher's XCD rotation and can split a plane over XCDs, whose
// L2s are not coherent with each other.  Each work-group therefore sets its
// hardware XCC id's bit in a per-plane mask at system scope before the first
// grid barrier (which also runs at system scope), and the plane then runs in
// one of two modes:
//  - local: every work-group on one XCD.  They share its L2: plain stores,
//    complete once they reach it, and agent-scope loads (which miss the CU's
//    L1 and read the L2) exchange the data, and a barrier is a plain flag
//    store and an agent-scope poll.
//  - fenced: the plane spans XCDs.  Stores and loads are agent-scope atomics,
//    and every barrier is a release fence (L2 write-back) before a
//    system-scope flag store and an acquire fence (cache invalidation) after
//    a system-scope poll.
// A work-group arrives at a barrier only after its own stores have completed
// (s_waitcnt 0).
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
__device__ inline void put(double *p, double v, bool local) {
    if (local) *p = v;
    else st_c(p, v);
}
__device__ inline void put2(double2 *p, double2 v, bool local) {
    if (local) *p = v;
    else st_c2(p, v);
}
// The XCC (XCD) this wave runs on.
__device__ inline int xcc_id() { return (int)(__builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xf); }
__device__ inline void st_sys2(double2 *p, double2 v) {
    __hip_atomic_store((double *)p, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store((double *)p + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline double2 ld_sys2(const double2 *p) {
    return make_double2(
        __hip_atomic_load(const_cast<double *>((const double *)p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM),
        __hip_atomic_load(const_cast<double *>((const double *)p + 1), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_SYSTEM));
}
enum BarMode { kBarSystem, kBarFenced, kBarLocal };
// Grid barrier among the W work-groups of one plane: work-group w publishes
// the number of barriers it has reached in its own flag, and lanes 0..W-1 of
// the first wave each wait for one work-group's flag, so no single counter is
// contended.  Returns false if the wait timed out (the caller then exits).
__device__ inline int load_flag(const int *p, BarMode mode) {
    int *q = const_cast<int *>(p);
    return mode == kBarLocal ? __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline bool plane_barrier(int *flags, int w, int W, int step, int *abort_s, int *status,
                                     BarMode mode) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (mode == kBarLocal) {
            flags[w] = step;
        } else {
            if (mode == kBarFenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(flags + w, step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    if ((int)threadIdx.x < W) {
        int spins = 0;
        while (load_flag(flags + threadIdx.x, mode) < step) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1 << 23)) {
                *abort_s = 1;
                atomicOr(status, kStatusBarrier);
                break;
            }
        }
    }
    __syncthreads();
    if (mode == kBarFenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *abort_s == 0;
}

// Reflector of the unblocked Hermitian reduction (LAPACK's elementary
// reflector convention): H^H x = (beta, 0, ...)^T, H = I - tau v v^H, v_0 = 1.
// x = col[k+1 .. F); computed identically by every work-group.  nrm_part is
// this thread's share of |x_2..|^2 (its rows >= k+2); the sum's barriers also
// publish col.
__device__ inline void reflector(const double2 *col, int k, int F, double *red, double2 *v,
                                 double2 &tk, double &beta, double nrm_part) {
    const double nrm = bsum(nrm_part, red);
    const double2 alpha = col[k + 1];
    tk = make_double2(0.0, 0.0);
    beta = alpha.x;
    double2 scale = make_double2(0.0, 0.0);
    if (nrm > 0.0 || alpha.y != 0.0) {
        beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + nrm), alpha.x);
        const double ib = 1.0 / beta;
        tk = make_double2((beta - alpha.x) * ib, -alpha.y * ib);
        const double2 den = make_double2(alpha.x - beta, alpha.y);
        const double idd = 1.0 / (den.x * den.x + den.y * den.y);
        scale = make_double2(den.x * idd, -den.y * idd);
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
    const int plane = a.plane0 + xcd + 8 * (slot / W), w = slot % W;
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
    __shared__ double2 wpart2[2][kCoopWaves];
    __shared__ int abort_s;
    if (t == 0) abort_s = 0;

    const double2 *C = a.C + (size_t)plane * F * F;
    double2 *H = a.H + (size_t)plane * F * F;
    double2 *tau = a.tau + (size_t)plane * F;
    double *d = a.d + (size_t)plane * F, *e = a.e + (size_t)plane * F;
    // double-buffered exchange areas (by step parity): p and the next column
    double2 *pbuf = a.pbuf + (size_t)plane * 2 * F;
    double2 *cbuf = a.vbuf + (size_t)plane * 2 * F;
    int *flags = a.bar + (size_t)plane * kBarStride;
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
    if (t == 0) {
        if (bad > 0.0) __hip_atomic_fetch_or(a.flag + plane, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_fetch_or(flags + kPlaceWord, 1 << xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // the owner of column 0 publishes it, in the odd-step half of the exchange
    // area: step 0 writes column 1 into the even half while a work-group that
    // passed the first barrier late may still be reading column 0.  This first
    // exchange and barrier run at system scope: the mode is not known yet.
    if (w == 0)
        for (int i = t; i < F; i += kCoopThreads) st_sys2(cbuf + F + i, Acol[i]);
    if (!plane_barrier(flags, w, W, ++nbar, &abort_s, a.status, kBarSystem)) return;
    if (__hip_atomic_load(a.flag + plane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
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
    const unsigned xccs =
        (unsigned)__hip_atomic_load(flags + kPlaceWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const bool local = !a.agent_scope && __popc(xccs) == 1;
    const BarMode bmode = local ? kBarLocal : kBarFenced;
    // thread t owns rows t + 256 m of the column being reduced (scol) and of
    // sv, sp; nrm_part is its share of the next reflector's |x|^2
    double nrm_part = 0.0;
    for (int i = t; i < F; i += kCoopThreads) {
        const double2 x = ld_sys2(cbuf + F + i);
        scol[i] = x;
        if (i >= 2) nrm_part += x.x * x.x + x.y * x.y;
    }

    double a2r = 0.0;   // 2 Re(alpha) of the pending rank-2 update (step k-1)
    for (int k = 0; k + 1 < F; ++k) {
        const int par = k & 1;
        // column k, with every update through step k-1 applied: its reflector
        double2 tk;
        double beta;
        reflector(scol, k, F, red, svn, tk, beta, nrm_part);
        __syncthreads();
        if (w == k % W) {
            for (int i = k + 1 + t; i < F; i += kCoopThreads) put2(H + (size_t)k * F + i, svn[i], local);
            if (t == 0) {
                put(d + k, scol[k].x, local);
                put(e + k, beta, local);
                put2(tau + k, tk, local);
            }
        }
        // own columns j > k: pending update, then p_j = tau_k sum_i conj(A[i][j]) v_i
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
            if (lane == 0) put2(pbuf + par * F + j, pj, local);
            if (j == k + 1)    // publish the next column (rows > k) for every work-group
                for (int i = k + 1 + lane; i < F; i += 64) put2(cbuf + par * F + i, col[i], local);
        }
        if (!plane_barrier(flags, w, W, ++nbar, &abort_s, a.status, bmode)) return;
        // every work-group reads all of p and the next column, forms p^H v itself
        // and applies the update of step k to column k+1 (rows > k)
        constexpr int kOwn = 64 * kCoopRows / kCoopThreads;     // rows per thread: F <= 512
        double2 pv[kOwn], cv[kOwn];
        const double2 pk1 = ld_c2(pbuf + par * F + k + 1);
#pragma unroll
        for (int m = 0; m < kOwn; ++m) {
            // all loads issued before any is used (rows <= k read a valid, unused slot)
            const int i = t + kCoopThreads * m, ii = (i > k && i < F) ? i : F - 1;
            pv[m] = ld_c2(pbuf + par * F + ii);
            cv[m] = ld_c2(cbuf + par * F + ii);
        }
        double ppr = 0.0, ppi = 0.0;
#pragma unroll
        for (int m = 0; m < kOwn; ++m) {
            const int i = t + kCoopThreads * m;
            if (i >= F) break;
            const bool live = i > k;
            const double2 vi = live ? svn[i] : make_double2(0.0, 0.0);
            if (live) {
                const double2 dv = cjmul2(pv[m], vi);
                ppr += dv.x;
                ppi += dv.y;
            }
            sv[i] = vi;
            sp[i] = live ? pv[m] : make_double2(0.0, 0.0);
        }
        const double2 pvh = bsum2(ppr, ppi, wpart);     // its syncs also publish sp and sv
        // alpha = -1/2 tau (p^H v); the pending update uses 2 Re(alpha)
        const double2 al = cmul2(make_double2(-0.5 * tk.x, -0.5 * tk.y), pvh);
        a2r = 2.0 * al.x;
        const double2 cpk = make_double2(pk1.x, -pk1.y), cvk = make_double2(svn[k + 1].x, -svn[k + 1].y);
        nrm_part = 0.0;
#pragma unroll
        for (int m = 0; m < kOwn; ++m) {
            const int i = t + kCoopThreads * m;
            if (i >= F) break;
            if (i > k) {
                const double2 x = pending(cv[m], sv[i], sp[i], cpk, cvk, a2r);
                scol[i] = x;
                if (i >= k + 3) nrm_part += x.x * x.x + x.y * x.y;
            }
        }
    }
    // last diagonal entry: column F-1 with the update of step F-2 applied
    __syncthreads();
    if (w == 0 && t == 0) {
        put(d + F - 1, scol[F - 1].x, local);
        put(e + F - 1, 0.0, local);
        put2(tau + F - 1, make_double2(0.0, 0.0), local);
    }
    if (!plane_barrier(flags, w, W, ++nbar, &abort_s, a.status, bmode)) return;

    // 2. every eigenvalue by multisection on Sturm counts: a group of kPoints
    //    lanes per eigenvalue counts at kPoints interior points of its bracket,
    //    so each round narrows the bracket (kPoints + 1)-fold
    double *sd = (double *)lds2;
    double *se2 = sd + F;
    double *se = se2 + F;
    double lo_b = 1e300, hi_b = -1e300, emax = 0.0;
    for (int i = t; i < F; i += kCoopThreads) {
        const double di = ld_c(d + i), ei = (i + 1 < F) ? ld_c(e + i) : 0.0;
        const double em = (i > 0) ? ld_c(e + i - 1) : 0.0;
        const double r = fabs(em) + fabs(ei);
        lo_b = fmin(lo_b, di - r);
        hi_b = fmax(hi_b, di + r);
        sd[i] = di;
        se[i] = ei;
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
    {
        // wave gw bisects eigenvalues kGroups gw + g (g = lane / kPoints): the
        // kPoints lanes of a group count at kPoints interior points of its
        // bracket, so each round narrows it (kPoints + 1)-fold
        const int gw = w * kCoopWaves + wave;
        const int g = lane / kPoints, pi = lane % kPoints;
        const int idx = gw * kGroups + g;
        const bool mine = idx < F;
        const int target = F - 1 - idx;                   // eigenvalues below this one
        double lo = lo_b, hi = hi_b;
        bool act = mine;
        for (int it = 0; it < 200; ++it) {
            if (act && hi - lo <= 2.0 * DBL_EPSILON * tnorm) act = false;
            if (__ballot(act) == 0ull) break;
            const double x = lo + (hi - lo) * (double)(pi + 1) / (double)(kPoints + 1);
            double q = sd[0] - x;
            int cnt = q < 0.0;
#pragma unroll 4
            for (int i = 1; i < F; ++i) {
                if (fabs(q) <= pivmin) q = -pivmin;
                // e2 / q through the hardware reciprocal and one Newton step
                // (within an ulp or two: the count is a sign test, and the
                // bracket ends at 2 eps |T| anyway)
                const double r0 = __builtin_amdgcn_rcp(q);
                const double rq = fma(r0, fma(-q, r0, 1.0), r0);
                q = (sd[i] - x) - se2[i - 1] * rq;
                cnt += q < 0.0;
            }
            // counts grow with x: the eigenvalue lies between the last point
            // below and the first point above
            const unsigned long long m = __ballot(cnt > target);
            const unsigned bits = (unsigned)((m >> (g * kPoints)) & ((1ull << kPoints) - 1ull));
            const int first = bits ? __ffs(bits) - 1 : kPoints;
            const double nlo = __shfl(x, g * kPoints + (first > 0 ? first - 1 : 0));
            const double nhi = __shfl(x, g * kPoints + (first < kPoints ? first : kPoints - 1));
            const double lo2 = first > 0 ? nlo : lo, hi2 = first < kPoints ? nhi : hi;
            if (act && lo2 == lo && hi2 == hi) act = false;
            if (act) {
                lo = lo2;
                hi = hi2;
            }
        }
        if (mine && pi == 0) {
            put(lam + idx, 0.5 * (lo + hi), local);
            if (a.lam_out) a.lam_out[(size_t)plane * F + idx] = 0.5 * (lo + hi);
        }
    }
    if (!plane_barrier(flags, w, W, ++nbar, &abort_s, a.status, bmode)) return;
    if (c <= 0) return;

    // 3. inverse iteration for eigenvector vi of T (the vi-th largest
    //    eigenvalue), work-group vi mod W, one thread: partial-pivoting LU of
    //    T - lambda I in LDS, three solves with recurrences carried in registers
    double *ts = a.tscr + (size_t)plane * c * 6 * F;
    double *__restrict__ u0 = se + F;
    double *__restrict__ u1 = u0 + F;
    double *__restrict__ u2 = u1 + F;
    double *__restrict__ ml = u2 + F;
    double *__restrict__ iu = ml + F;
    double *__restrict__ sw = iu + F;
    double *__restrict__ y = sw + F;
    for (int vi = w; vi < c; vi += W) {
        // the start vector, by every thread (the factor and solves below are
        // serial recurrences, run by thread 0)
        for (int i = t; i < F; i += kCoopThreads) y[i] = 1.0 + 0.37 * sin(0.731 * i + 1.3 * vi);
        __syncthreads();
        if (t == 0) {
            const double lm = ld_c(lam + vi);
            const double tiny = DBL_EPSILON * tnorm + pivmin;
            // factor: rows i, i+1 enter step i as (c0, c1 | sub) over (next0, next1)
            double c0 = sd[0] - lm, c1 = F > 1 ? se[0] : 0.0;
#pragma unroll 4
            for (int i = 0; i + 1 < F; ++i) {
                const double sub = se[i];
                double n0 = sd[i + 1] - lm;
                double n1 = (i + 2 < F) ? se[i + 1] : 0.0;
                double m2 = 0.0, mul;
                bool swp;
                if (fabs(c0) >= fabs(sub)) {
                    if (c0 == 0.0) c0 = tiny;
                    mul = sub / c0;
                    n0 -= mul * c1;
                    swp = false;
                } else {
                    mul = c0 / sub;
                    const double t1 = n0, t2 = n1;
                    c0 = sub;
                    n0 = c1 - mul * t1;
                    n1 = -mul * t2;
                    c1 = t1;
                    m2 = t2;
                    swp = true;
                }
                u0[i] = c0;
                u1[i] = c1;
                u2[i] = m2;
                ml[i] = mul;
                iu[i] = 1.0 / c0;
                sw[i] = swp ? 1.0 : 0.0;
                c0 = n0;
                c1 = n1;
            }
            if (c0 == 0.0) c0 = tiny;
            u0[F - 1] = c0;
            u1[F - 1] = 0.0;
            u2[F - 1] = 0.0;
            iu[F - 1] = 1.0 / c0;
            for (int it = 0; it < 3; ++it) {
                // forward: apply the row swaps and multipliers
                double cur = y[0];
#pragma unroll 4
                for (int i = 0; i + 1 < F; ++i) {
                    const double nxt = y[i + 1];
                    const bool swp = sw[i] != 0.0;
                    const double top = swp ? nxt : cur;
                    const double bot = swp ? cur : nxt;
                    y[i] = top;
                    cur = bot - ml[i] * top;
                }
                y[F - 1] = cur;
                // back substitution
                double x1 = y[F - 1] * iu[F - 1], x2 = 0.0;
                y[F - 1] = x1;
                double n2 = x1 * x1;
#pragma unroll 4
                for (int i = F - 2; i >= 0; --i) {
                    const double xi = (y[i] - u1[i] * x1 - u2[i] * x2) * iu[i];
                    y[i] = xi;
                    n2 += xi * xi;
                    x2 = x1;
                    x1 = xi;
                }
                const double inv = 1.0 / sqrt(n2);
                for (int i = 0; i < F; ++i) y[i] *= inv;
            }
            double *yo = ts + (size_t)vi * 6 * F + 4 * F;
            for (int i = 0; i < F; ++i) put(yo + i, y[i], local);
        }
        __syncthreads();
    }
    if (!plane_barrier(flags, w, W, ++nbar, &abort_s, a.status, bmode)) return;

    // 4. work-group 0: two passes of classical Gram-Schmidt over the c vectors
    //    (staged in LDS), then normalise
    if (w == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double *Y = se + F;                            // [c][F]
        double *gdot = Y + (size_t)c * F;              // [c]
        for (int i = t; i < c * F; i += kCoopThreads)
            Y[i] = ts[(size_t)(i / F) * 6 * F + 4 * F + (i % F)];
        __syncthreads();
        for (int i = 0; i < c; ++i) {
            double *bi = Y + (size_t)i * F;
            for (int pass = 0; pass < 2; ++pass) {
                for (int j = wave; j < i; j += kCoopWaves) {
                    const double *bj = Y + (size_t)j * F;
                    double s = 0.0;
                    for (int q = lane; q < F; q += 64) s += bj[q] * bi[q];
                    s = wsum(s);
                    if (lane == 0) gdot[j] = s;
                }
                __syncthreads();
                for (int q = t; q < F; q += kCoopThreads) {
                    double x = bi[q];
                    for (int j = 0; j < i; ++j) x -= gdot[j] * Y[(size_t)j * F + q];
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
        for (int i = t; i < c * F; i += kCoopThreads)
            put(ts + (size_t)(i / F) * 6 * F + 4 * F + (i % F), Y[i], local);
    }
    if (!plane_barrier(flags, w, W, ++nbar, &abort_s, a.status, bmode)) return;

    // 5. back-transformation x = H_0 H_1 ... H_{F-2} y: work-group w forms
    //    vectors w, w + W, ...; thread t holds rows t + 256 m of x, the wave sums
    //    meet in LDS (double-buffered by step parity, one barrier per step), and
    //    the Householder rows of the next three steps are in flight
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double2 *V = a.V + (size_t)plane * F * c;
    constexpr int kOwn = 64 * kCoopRows / kCoopThreads;     // rows per thread: F <= 512
    int bpar = 0;
    for (int vi = w; vi < c; vi += W) {
        const double *y = ts + (size_t)vi * 6 * F + 4 * F;
        double2 x[kOwn];
#pragma unroll
        for (int m = 0; m < kOwn; ++m) {
            const int q = t + kCoopThreads * m;
            x[m] = make_double2(q < F ? y[q] : 0.0, 0.0);
        }
        auto fetch = [&](int k, double2 (&h)[kOwn], double2 &tk) {
            tk = k >= 0 ? tau[k] : make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < kOwn; ++m) {
                const int q = t + kCoopThreads * m;
                h[m] = (k >= 0 && q > k && q < F) ? H[(size_t)k * F + q] : make_double2(0.0, 0.0);
            }
        };
        double2 h0[kOwn], h1[kOwn], h2[kOwn], h3[kOwn], t0, t1, t2, t3;
        fetch(F - 2, h0, t0);
        fetch(F - 3, h1, t1);
        fetch(F - 4, h2, t2);
        for (int k = F - 2; k >= 0; --k) {
            fetch(k - 3, h3, t3);
            if (t0.x != 0.0 || t0.y != 0.0) {          // the same for every thread
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int m = 0; m < kOwn; ++m) {
                    const double2 p = cjmul2(h0[m], x[m]);
                    sr += p.x;
                    si += p.y;
                }
                sr = wsum(sr);
                si = wsum(si);
                if (lane == 0) wpart2[bpar][wave] = make_double2(sr, si);
                __syncthreads();
                double2 tot = make_double2(0.0, 0.0);
#pragma unroll
                for (int i = 0; i < kCoopWaves; ++i) {
                    tot.x += wpart2[bpar][i].x;
                    tot.y += wpart2[bpar][i].y;
                }
                bpar ^= 1;
                const double2 sc = cmul2(t0, tot);
#pragma unroll
                for (int m = 0; m < kOwn; ++m) {
                    const double2 p = cmul2(h0[m], sc);
                    x[m] = make_double2(x[m].x - p.x, x[m].y - p.y);
                }
            }
#pragma unroll
            for (int m = 0; m < kOwn; ++m) {
                h0[m] = h1[m];
                h1[m] = h2[m];
                h2[m] = h3[m];
            }
            t0 = t1;
            t1 = t2;
            t2 = t3;
        }
#pragma unroll
        for (int m = 0; m < kOwn; ++m) {
            const int q = t + kCoopThreads * m;
            if (q < F) V[(size_t)q * c + vi] = x[m];
        }
    }
}

int eigen_coop_width(int F) { return std::max(1, std::min(kCoopMaxW, cdiv(F, 10))); }

size_t eigen_coop_lds(int F, int c) {
    if (F > 64 * kCoopRows || F > kGroups * kCoopWaves * eigen_coop_width(F)) return SIZE_MAX;
    const int W = eigen_coop_width(F);
    // reduction: own columns + 4 vectors; tail: d, e^2 and either the six LU
    // arrays or the c Gram-Schmidt vectors plus their dots
    const size_t red_b = ((size_t)cdiv(F, W) * F + 4 * (size_t)F) * sizeof(double2);
    const size_t tail_b = (3 * (size_t)F + std::max((size_t)7 * F, (size_t)c * F + c)) * sizeof(double);
    return std::max(red_b, tail_b) + 64 * sizeof(double);
}

// A cooperative launch needs every work-group resident at once, so the planes
// are solved in groups: as many whole rounds of 8 planes (one per XCD) as fit.
hipError_t launch_eigen_coop(const EigArgs &args, hipStream_t st) {
    const unsigned lds = (unsigned)eigen_coop_lds(args.F, args.c);
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)eigen_coop_kernel,
                                                         kCoopThreads, lds);
    if (e != hipSuccess) return e;
    const int resident = per_cu * ncu;
    const int group = resident / (8 * args.W) * 8;           // whole rounds of 8 planes
    if (group == 0) return hipErrorCooperativeLaunchTooLarge;
    for (int p0 = 0; p0 < args.planes; p0 += group) {
        EigArgs a = args;
        a.plane0 = p0;
        a.planes = std::min(args.planes, p0 + group);        // planes [p0, a.planes)
        const int n = a.planes - p0;
        dim3 grid(8 * cdiv(n, 8) * args.W), block(kCoopThreads);
        void *params[] = {&a};
        e = hipLaunchCooperativeKernel((const void *)eigen_coop_kernel, grid, block, params, lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ulm
