// Projected Tikhonov problem of RTG-GMRES in float64, one workgroup per
// problem (eqs. (12)-(13), with mu fixed or chosen by the discrepancy
// principle).
//
// The Arnoldi steps already reduced H (the (k+1) x k Hessenberg matrix) by
// Givens rotations to H = Q [R; 0] with Q^T beta e1 = [g_R; gamma], so
//   ||beta e1 - H y||^2 + mu ||y||^2 = ||g_R - R y||^2 + gamma^2 + mu ||y||^2.
// With the SVD R = U diag(s) W^T (one-sided Jacobi: plane rotations of the
// columns of R accumulated in W, in LDS) and ghat = U^T g_R,
//   phi(mu) = sum_i (mu / (s_i^2 + mu))^2 ghat_i^2 + gamma^2
// is the projected residual; it increases from gamma^2 to beta^2 and the
// discrepancy principle takes the root of phi(mu) = (eta delta)^2, found by
// multisection (64 points per pass) in log(mu).  Then y = W diag(s / (s^2 + mu)) ghat, the filter
// form of the stacked least-squares problem (13).  With the GCV rule (Sec. 3,
// parameter selection via GCV) mu minimises
//   GCV(mu) = phi(mu) / (1 + sum_i mu / (s_i^2 + mu))^2
// (the trace of I - H (H^T H + mu I)^{-1} H^T over the k + 1 rows): the best
// of 512 points spread over [log s_min^2 - 10, log s_max^2 + 10], then passes
// of 64 points between the neighbours of the best point so far.  The kernel
// writes the coefficients -y_j of the solution update and the result summary.
#include "rtg_internal.h"

namespace rtg {

// A pair of columns counts as orthogonal once |a_p . a_q| <= tol ||a_p|| ||a_q||;
// below about n * eps the inner product is rounding noise and rotations stop
// making progress.
constexpr double JACOBI_TOL = 1e-13;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// phi(mu) evaluated by one wave (k <= 128 terms, two per lane)
__device__ __forceinline__ double proj_res2(const double* sig, const double* gh, int k, double mu,
                                            double gp2, int lane) {
    double s = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double f = mu / (sig[i] * sig[i] + mu);
        s += f * f * gh[i] * gh[i];
    }
    return wave_sum(s) + gp2;
}

__global__ void __launch_bounds__(1024) k_solve(const Desc* __restrict__ descs) {
    constexpr int LD = MMAX + 1;
    __shared__ double As[MMAX * LD];
    __shared__ double Ws[MMAX * LD];
    __shared__ double gR[MMAX], sig[MMAX], gh[MMAX], fco[MMAX];
    __shared__ int s_rot;
    __shared__ double s_mu;
    __shared__ int s_flags;

    const Desc& d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwave = blockDim.x >> 6;
    const int k = d.state[ST_MEFF];
    const int m = d.m;
    const double beta = d.scal[SC_BETA];
    const double* gvec = d.gv + 2 * m;

    if (d.state[ST_SKIP]) return;         // a restart cycle this problem sits out
    const int done = d.state[ST_ITERS];   // steps of earlier restart cycles
    if (k == 0) {
        if (tid == 0) {
            d.coef[MMAX + 1] = 1.f;
            rtg_info inf;
            inf.iters = done;
            inf.flags = d.state[ST_FLAGS];
            inf.mu = 0.0;
            inf.beta = beta;
            inf.res_proj = beta;
            inf.res_ls = beta;
            *d.info = inf;
        }
        return;
    }
    // ---- load R (upper triangular, column-major, leading dimension m) and W = I
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int c = e / k, r = e % k;
        As[c * LD + r] = (r <= c) ? d.R[(size_t)c * m + r] : 0.0;
        Ws[c * LD + r] = (r == c) ? 1.0 : 0.0;
    }
    if (tid < k) gR[tid] = gvec[tid];
    const double gam = fabs(gvec[k]);
    __syncthreads();

    // ---- one-sided Jacobi, round-robin (circle) ordering of column pairs.
    // Sixteen lanes handle one pair (k <= 96: at most six rows per lane), so
    // all pairs of a round (k/2 <= 48 <= 64 groups) rotate concurrently.
    const int nb = k + (k & 1);
    const int grp = tid >> 4, gl = tid & 15, ngrp = blockDim.x >> 4;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int rd = 0; rd < nb - 1; ++rd) {
            for (int pi = grp; pi < nb / 2; pi += ngrp) {
                const int pos_b = nb - 1 - pi;
                const int pa = pi == 0 ? 0 : 1 + (pi - 1 + rd) % (nb - 1);
                const int pb = 1 + (pos_b - 1 + rd) % (nb - 1);
                if (pa >= k || pb >= k) continue;      // uniform within the 16-lane group
                double* ca = As + pa * LD;
                double* cb = As + pb * LD;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = gl; r < k; r += 16) {
                    const double x = ca[r], y = cb[r];
                    al += x * x; be += y * y; ga += x * y;
                }
#pragma unroll
                for (int off = 8; off > 0; off >>= 1) {
                    al += __shfl_xor(al, off, 16);
                    be += __shfl_xor(be, off, 16);
                    ga += __shfl_xor(ga, off, 16);
                }
                if (ga != 0.0 && fabs(ga) > JACOBI_TOL * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cth = 1.0 / sqrt(1.0 + t * t), sth = cth * t;
                    double* wa = Ws + pa * LD;
                    double* wb = Ws + pb * LD;
                    for (int r = gl; r < k; r += 16) {
                        const double x = ca[r], y = cb[r];
                        ca[r] = cth * x - sth * y;
                        cb[r] = sth * x + cth * y;
                        const double u = wa[r], v = wb[r];
                        wa[r] = cth * u - sth * v;
                        wb[r] = sth * u + cth * v;
                    }
                    if (gl == 0) s_rot = 1;
                }
            }
            __syncthreads();
        }
        const int rot = s_rot;
        __syncthreads();
        if (!rot) break;
    }
    // ---- singular values and ghat = U^T g_R
    for (int i = wave; i < k; i += nwave) {
        double nn = 0.0, gg = 0.0;
        for (int r = lane; r < k; r += 64) {
            const double x = As[i * LD + r];
            nn += x * x;
            gg += x * gR[r];
        }
        nn = wave_sum(nn);
        gg = wave_sum(gg);
        if (lane == 0) {
            const double s = sqrt(nn);
            sig[i] = s;
            gh[i] = s > 0.0 ? gg / s : 0.0;
        }
    }
    __syncthreads();
    // ---- mu: fixed, or the discrepancy principle (wave 0)
    if (wave == 0) {
        const double gp2 = gam * gam;
        double mu = d.mu;
        int flags = 0;
        if (!d.mu_fixed && d.mu_rule == RTG_MU_GCV) {
            // GCV at log(mu) = x, and the (value, position) minimum over the wave
            auto gcv_at = [&](double x) {
                const double mu_l = exp(x);
                double ph = gp2, tr = 1.0;
                for (int i = 0; i < k; ++i) {
                    const double s2 = sig[i] * sig[i];
                    const double f = mu_l / (s2 + mu_l);
                    ph += f * f * gh[i] * gh[i];
                    tr += s2 > 0.0 ? f : 1.0;
                }
                return ph / (tr * tr);
            };
            auto wave_argmin = [&](double v, int idx, double& vmin, int& imin) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(v, off, 64);
                    const int oi = __shfl_xor(idx, off, 64);
                    if (ov < v || (ov == v && oi < idx)) { v = ov; idx = oi; }
                }
                vmin = v;
                imin = idx;
            };
            double smax = 0.0, smin = INFINITY;
            for (int i = lane; i < k; i += 64) {
                smax = fmax(smax, sig[i]);
                if (sig[i] > 0.0) smin = fmin(smin, sig[i]);
            }
            smax = wave_max(smax);
            smin = -wave_max(-smin);
            const double smax2 = smax > 0.0 ? smax * smax : 1.0;
            const double smin2 = isfinite(smin) ? fmax(smin * smin, 1e-30 * smax2) : smax2;
            const double glo = log(smin2) - 10.0, ghi = log(smax2) + 10.0;
            // 512 grid points, eight per lane (the same grid as the oracle's)
            double bv = INFINITY;
            int bi = 0;
            for (int q = 0; q < 8; ++q) {
                const int pidx = 8 * lane + q;
                const double v = gcv_at(glo + (ghi - glo) * (double)pidx / 511.0);
                if (v < bv) { bv = v; bi = pidx; }
            }
            double vmin;
            int imin;
            wave_argmin(bv, bi, vmin, imin);
            double lo = glo + (ghi - glo) * (double)max(imin - 1, 0) / 511.0;
            double hi = glo + (ghi - glo) * (double)min(imin + 1, 511) / 511.0;
            double xbest = glo + (ghi - glo) * (double)imin / 511.0;
            for (int it = 0; it < 16; ++it) {
                const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
                double v = gcv_at(x);
                if (!(v < vmin)) v = INFINITY;            // keep the best point so far when nothing beats it
                int li;
                double lv;
                wave_argmin(v, lane, lv, li);
                if (!(lv < INFINITY)) {                  // the best point is inside a bracket no lane improves:
                    const double w = (hi - lo) / 65.0;   // shrink around it
                    lo = fmax(lo, xbest - w);
                    hi = fmin(hi, xbest + w);
                } else {
                    vmin = lv;
                    xbest = lo + (hi - lo) * (double)(li + 1) / 65.0;
                    const double w = (hi - lo) / 65.0;
                    lo = xbest - w;
                    hi = xbest + w;
                }
                if (!(hi - lo > 1e-12)) break;
            }
            mu = exp(xbest);
        } else if (!d.mu_fixed) {
            const double t = d.eta * d.delta;
            const double t2 = t * t;
            if (t2 <= gp2) {
                mu = 0.0;
                flags |= RTG_F_DISCREP_UNREACHABLE;
            } else if (t2 >= beta * beta) {
                mu = INFINITY;
                flags |= RTG_F_MU_INF;
            } else {
                double smax = 0.0;
                for (int i = lane; i < k; i += 64) smax = fmax(smax, sig[i]);
                smax = wave_max(smax);
                const double smax2 = smax > 0.0 ? smax * smax : 1.0;
                double lo = log(smax2) - 80.0, hi = log(smax2) + 80.0;
                for (int it = 0; it < 40 && proj_res2(sig, gh, k, exp(lo), gp2, lane) > t2; ++it) lo -= 40.0;
                for (int it = 0; it < 40 && proj_res2(sig, gh, k, exp(hi), gp2, lane) < t2; ++it) hi += 40.0;
                // Multisection in log(mu): each lane evaluates phi at one of 64
                // interior points of [lo, hi]; phi increases with mu, so the
                // lanes below the target form a prefix and the bracket shrinks
                // 65-fold per pass (the bracket bisection would reach, six
                // halvings at a time), until it stops shrinking.
                for (int it = 0; it < 16; ++it) {
                    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
                    double ph = gp2;
                    const double mu_l = exp(x);
                    for (int i = 0; i < k; ++i) {
                        const double f = mu_l / (sig[i] * sig[i] + mu_l);
                        ph += f * f * gh[i] * gh[i];
                    }
                    const unsigned long long below = __ballot(ph < t2);
                    const int pfx = (below == ~0ull) ? 64 : __builtin_ctzll(~below);
                    const double nlo = pfx > 0 ? __shfl(x, pfx - 1, 64) : lo;
                    const double nhi = pfx < 64 ? __shfl(x, pfx, 64) : hi;
                    if (!(nhi - nlo < hi - lo)) break;
                    lo = nlo;
                    hi = nhi;
                }
                mu = exp(0.5 * (lo + hi));
            }
        }
        if (lane == 0) {
            s_mu = mu;
            s_flags = flags;
        }
    }
    __syncthreads();
    const double mu = s_mu;
    if (tid < k) {
        const double s = sig[tid];
        fco[tid] = isinf(mu) ? 0.0 : (s > 0.0 ? s / (s * s + mu) * gh[tid] : 0.0);
    }
    __syncthreads();
    // ---- y = W f; coefficients of X = X0 + sum_j y_j V_j
    bool ok = true;
    if (tid < k) {
        double yv = 0.0;
        for (int i = 0; i < k; ++i) yv += Ws[i * LD + tid] * fco[i];
        d.y[tid] = yv;
        // (a V_1 stored unnormalised carries its 1 / beta in its coefficient)
        d.coef[tid] = (float)(-yv * ((d.lazy_v1 && tid == 0) ? 1.0 / beta : 1.0));
        ok = isfinite(yv);
    }
    const int allok = __syncthreads_and(ok ? 1 : 0);
    if (wave == 0) {
        const double gp2 = gam * gam;
        const double rp2 = isinf(mu) ? beta * beta : proj_res2(sig, gh, k, mu, gp2, lane);
        if (lane == 0) {
            int flags = d.state[ST_FLAGS] | s_flags;
            if (!allok) flags |= RTG_F_NONFINITE;
            d.state[ST_FLAGS] = flags;
            d.coef[MMAX + 1] = 1.f;
            d.scal[SC_MU] = mu;
            d.scal[SC_RESPROJ] = sqrt(rp2);
            d.state[ST_ITERS] = done + k;
            rtg_info inf;
            inf.iters = done + k;
            inf.flags = flags;
            inf.mu = mu;
            inf.beta = beta;
            inf.res_proj = sqrt(rp2);
            inf.res_ls = gam;
            *d.info = inf;
        }
    }
}

// cycle 0: a fresh solve.  cycle c > 0 (restarted RTG-GMRES): a new cycle
// from X0 = X; a problem out of restarts, or one that sat out an earlier
// cycle (its residual was below eps), sits this one out too; the others
// keep their step count and flags (but for NOT_CONVERGED, which the cycle
// decides anew).
__global__ void k_init(const Desc* __restrict__ descs, int cycle, int* sched) {
    const Desc& d = descs[blockIdx.x];
    const int tid = threadIdx.x;
    if (sched && blockIdx.x == 0)
        for (int w = tid; w < SCH_WORDS; w += blockDim.x) sched[w] = 0;
    if (cycle > 0) {
        const bool sit_out = cycle > d.restarts || d.state[ST_SKIP] != 0;
        __syncthreads();                      // every thread has read the state
        if (sit_out) {
            if (tid == 0) {
                d.state[ST_SKIP] = 1;
                d.state[ST_ACTIVE] = 0;
            }
            if (tid < NKIND) d.state[ST_DONE + tid] = 0;
            return;
        }
        if (tid < NSTATE) {
            const int v = d.state[tid];
            int nv = 0;
            if (tid == ST_ACTIVE) nv = 1;
            else if (tid == ST_ITERS) nv = v;
            else if (tid == ST_FLAGS) nv = v & ~RTG_F_NOT_CONVERGED;
            d.state[tid] = nv;
        }
    } else if (tid < NSTATE) {
        d.state[tid] = (tid == ST_ACTIVE) ? 1 : ((tid == ST_FLAGS && d.fallback) ? RTG_F_FALLBACK : 0);
    }
    if (tid < NSCAL) d.scal[tid] = 0.0;
    if (tid == 0) d.coef[MMAX + 1] = 1.f;   // the scale of a V_1 formed before the start step
    const int m = d.m;
    for (int e = tid; e < (m + 1) * m; e += blockDim.x) d.H[e] = 0.0;
    for (int e = tid; e < 3 * m + 1; e += blockDim.x) d.gv[e] = 0.0;
}

// Composed sketch matrices: S(Phi(X)) = X x_1 (Om1 A1) x_2 (Om2 A2) x_3 (Om3 B^T)
// (mode products compose; Phi of eq. (2)).  Om1 is the matrix the basis
// sketches use: the bfloat16-rounded one for a bfloat16 basis.  A1 has band
// rows, A1[i', i] = a1[i' (2 r1 + 1) + r1 + i - i'] (read here from the
// transposed copy, so that neighbouring entries read neighbouring words);
// B[k, j] = bb[k (2 rB + 1) + rB + j - k]
// is the weight of input channel k in output channel j.
__global__ void k_compose(const Desc* __restrict__ descs, int nbc) {
    const int p = blockIdx.x / nbc, part = blockIdx.x % nbc;
    const Desc& d = descs[p];
    if (d.st != nullptr) return;          // a general PSF: no banded factors to compose
    const int I1 = d.I1, I2 = d.I2, J = d.J, l1 = d.l1, l2 = d.l2, l3 = d.l3;
    const int r1 = d.r1, r2 = d.r2, rB = d.rB;
    const int wB = 2 * rB + 1;
    // mode 1 over the operand-padded index space: padding entries are
    // written as zeros (the MFMA contractions read whole tiles)
    const int I1p = frag_nkb(I1, FRAG_K_BF16) * FRAG_K_BF16;
    const int E1 = (int)compose_mode1_entries(l1, I1), E2 = l2 * I2, E3 = l3 * J;
    const int nkf = frag_nkb(I1, FRAG_K_F32), nkh = frag_nkb(I1, FRAG_K_BF16);
    const size_t lo_plane = frag_elems(l1, I1, FRAG_K_BF16);
    // one entry per thread; taps read from clamped indices and masked, so
    // that the loads of a thread are independent of each other
    const int e = part * blockDim.x + threadIdx.x;
    if (e < E1) {
        const int a = e / I1p, i = e % I1p;
        const bool real = a < l1 && i < I1;
        const int ac = min(a, l1 - 1);
        float acc = 0.f;
#pragma unroll 5
        for (int dd = -r1; dd <= r1; ++dd) {
            const int ip = i - dd;
            const int ipc = min(max(ip, 0), I1 - 1);
            const float om = d.skbf ? bf2f(*gptr(d.om1h + (size_t)ac * I1 + ipc)) : *gptr(d.om1 + (size_t)ac * I1 + ipc);
            const float w = *gptr(d.a1t + (size_t)(r1 + dd) * I1 + ipc);
            acc = fmaf((ip >= 0 && ip < I1) ? om : 0.f, w, acc);
        }
        acc = real ? acc : 0.f;
        if (i < nkf * FRAG_K_F32) *gptr_w((float*)d.om1t + frag_index(a, i, nkf, FRAG_K_F32)) = acc;
        const bf16_t hi = f2bf(acc);
        const size_t fh = frag_index(a, i, nkh, FRAG_K_BF16);
        *gptr_w((bf16_t*)d.om1th + fh) = hi;
        *gptr_w((bf16_t*)d.om1th + lo_plane + fh) = f2bf(acc - bf2f(hi));
    } else if (e < E1 + E2) {
        const int e2 = e - E1;
        const int b = e2 / I2, i = e2 % I2;
        float acc = 0.f;
#pragma unroll 5
        for (int dd = -r2; dd <= r2; ++dd) {
            const int ip = i - dd;
            const int ipc = min(max(ip, 0), I2 - 1);
            const float om = *gptr(d.om2 + (size_t)b * I2 + ipc);
            const float w = *gptr(d.a2t + (size_t)(r2 + dd) * I2 + ipc);
            acc = fmaf((ip >= 0 && ip < I2) ? om : 0.f, w, acc);
        }
        *gptr_w((float*)d.om2t + e2) = acc;
    } else if (e < E1 + E2 + E3) {
        const int e3 = e - E1 - E2;
        const int c3 = e3 / J, k = e3 % J;
        float acc = 0.f;
        for (int j = max(0, k - rB); j <= min(J - 1, k + rB); ++j) {
            const float o3 = d.has_om3 ? *gptr(d.om3 + (size_t)c3 * J + j) : (c3 == j ? 1.f : 0.f);
            acc = fmaf(o3, *gptr(d.bb + (size_t)k * wB + rB + (j - k)), acc);
        }
        *gptr_w((float*)d.om3t + e3) = acc;
    }
}

__global__ void k_finish_arnoldi(const Desc* __restrict__ descs, double* H, double* beta,
                                 int* m_done, int m) {
    const Desc& d = descs[0];
    for (int e = threadIdx.x; e < (m + 1) * m; e += blockDim.x) H[e] = d.H[e];
    if (threadIdx.x == 0) {
        *beta = d.scal[SC_BETA];
        *m_done = d.state[ST_MEFF];
    }
}

hipError_t launch_solve(const Desc* d, int count, int mmax, hipStream_t s) {
    // sixteen lanes per Jacobi column pair; at least 128 threads (one per
    // column for the final products), so that small problems synchronise
    // few waves
    int threads = 16 * ((mmax + 1) / 2);
    threads = (threads + 63) / 64 * 64;
    threads = threads < 128 ? 128 : (threads > 1024 ? 1024 : threads);
    hipLaunchKernelGGL(k_solve, dim3(count), dim3(threads), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_init(const Desc* d, int count, hipStream_t s, int cycle, int* sched) {
    hipLaunchKernelGGL(k_init, dim3(count), dim3(256), 0, s, d, cycle, sched);
    return hipGetLastError();
}

hipError_t launch_compose(const Desc* d, int count, int max_entries, hipStream_t s) {
    const int nbc = (max_entries + 255) / 256;
    hipLaunchKernelGGL(k_compose, dim3(count * nbc), dim3(256), 0, s, d, nbc);
    return hipGetLastError();
}

hipError_t launch_finish_arnoldi(const Desc* d, double* H, double* beta, int* m_done, int m,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_finish_arnoldi, dim3(1), dim3(256), 0, s, d, H, beta, m_done, m);
    return hipGetLastError();
}

}  // namespace rtg
