#pragma once
// Sketched inner products and the Hessenberg update of one Arnoldi step.
//
// Each workgroup owns a chunk of (a, b) index pairs of the sketch.  It
//  1. finishes the sketch for its chunk: sums the per-tile partials written
//     by k_tile over the i2 tiles, and applies mode 3,
//        s[a,b,c'] = sum_c Om3[c',c] sum_tiles P_(tile,c)[a,b]
//     (Om3 = identity when absent) -- for s = S(Phi(V_j)) and, in a step,
//     for S(V_j), the sketch of the newest stored basis tensor.  In a step
//     the partials of s were taken from V_j with Om1 A1 and Om2 A2, and
//     mode 3 uses Om3 B^T (mode products compose);
//  2. computes its share of the inner products <S(V_i), s> and
//     <S(V_i), S(V_j)> (i <= j) and of ||s||^2 in float64;
//  3. the last workgroup of a problem to finish sums the shares in a fixed
//     order and performs the small, float64 part of the step (Sec. 4.3):
//        h1 = S(V)^T s,  h = h1 + (h1 - G h1)        (classical Gram-Schmidt
//                                                     with one reorthogonal-
//                                                     isation, G = S(V)^T S(V))
//        h_{j+1,j} = ||s - S(V) h|| = sqrt(||s||^2 - 2 h^T h1 + h^T G h)
//     then the breakdown test, the Givens update of the least-squares
//     problem (11S) and the stopping decision.  It writes the coefficients
//     for the next multi-AXPY (k_tile).
// In the start mode it returns beta = ||S(R0)||; in the sketch-output mode it
// writes the finished sketch in the column-major order of the C ABI.
//
// Golub-Kahan mode (Sec. 4.5): the newest tensor X_c of one side (V_c, or
// U_c on the side of Phi^T) was sketched with Omega and with the composed
// matrices of its side's operator, so s = S(Op(X_c)) is finished here as in
// a step, and the next coefficient of the bidiagonal matrix is
//   ||s - cf S(Y)||,  Y the other side's newest tensor, cf its coefficient
// (alpha_c = ||S(Phi^T(U_c)) - beta_c S(V_{c-1})|| on the U side,
//  beta_{c+1} = ||S(Phi(V_c)) - alpha_c S(U_c)|| on the V side),
// summed element by element in float64.  The V side completes column c of
// the bidiagonal matrix and takes the same Givens update and stopping
// decisions as a GMRES step.

#include "rtg_internal.h"

namespace rtg {

// largest step whose stored block of G the finishing workgroup stages in LDS
constexpr int GLDS = 64;

__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Finished sketch for the pairs [q0, q0 + qn):
//   out[(q - q0) l3 + c'] = sum_c M[c', c] sum_{i2 tiles t of channel c} P[(c, t)][q]
// with M = m3 (l3 x J) or the identity (m3 == nullptr); band >= 0 says that
// M[c', c] = 0 for |c' - c| > band.  NB buffers are finished together.
// Output channels are taken 16 at a time; three input channels at a time,
// their partials (16 tiles each, of every buffer) are loaded together, all
// in flight (clamped indices, masked), and summed in a fixed order.
template <int NB>
__device__ __forceinline__ void finish_sketches(const Desc& d, int q0, int qn,
                                                const float* __restrict__ P0, const float* __restrict__ m30,
                                                int band0, float* out0, const float* __restrict__ P1,
                                                const float* __restrict__ m31, int band1, float* out1) {
    constexpr int U = 16, G3 = 16, CP = 3;
    const int tid = block_tid();
    const int L12 = d.l1 * d.l2;
    const int J = d.J, nt2 = d.n_i2t, l3 = d.l3;
    // channels that feed output channels [g, g + G3)
    auto reach = [&](const float* m3, int band) { return m3 == nullptr ? 0 : (band >= 0 ? band : J); };
    const int rch = max(reach(m30, band0), NB > 1 ? reach(m31, band1) : 0);
    for (int t = tid; t < qn; t += blockDim.x) {
        const int q = q0 + t;
        for (int g = 0; g < l3; g += G3) {
            float a0[G3], a1[G3];
#pragma unroll
            for (int c3 = 0; c3 < G3; ++c3) { a0[c3] = 0.f; a1[c3] = 0.f; }
            const int clo = max(0, g - rch), chi = min(J, g + G3 + rch);
            for (int c0 = clo; c0 < chi; c0 += CP) {
                float Q0[CP], Q1[CP];
#pragma unroll
                for (int cc = 0; cc < CP; ++cc) { Q0[cc] = 0.f; Q1[cc] = 0.f; }
                for (int t20 = 0; t20 < nt2; t20 += U) {
                    float v0[CP][U], v1[CP][U];
#pragma unroll
                    for (int cc = 0; cc < CP; ++cc)
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int c = min(c0 + cc, chi - 1);
                            const size_t off = ((size_t)c * nt2 + min(t20 + u, nt2 - 1)) * L12 + q;
                            v0[cc][u] = *gptr(P0 + off);
                            if constexpr (NB > 1) v1[cc][u] = *gptr(P1 + off);
                        }
#pragma unroll
                    for (int cc = 0; cc < CP; ++cc)
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const bool ok = t20 + u < nt2;
                            Q0[cc] += ok ? v0[cc][u] : 0.f;
                            if constexpr (NB > 1) Q1[cc] += ok ? v1[cc][u] : 0.f;
                        }
                }
#pragma unroll
                for (int cc = 0; cc < CP; ++cc) {
                    const int c = c0 + cc;
                    if (c >= chi) break;
#pragma unroll
                    for (int c3 = 0; c3 < G3; ++c3) {
                        const int r = min(g + c3, l3 - 1);
                        const float w0 = m30 ? *gptr(m30 + (size_t)r * J + c) : (g + c3 == c ? 1.f : 0.f);
                        a0[c3] = fmaf(w0, Q0[cc], a0[c3]);
                        if constexpr (NB > 1) {
                            const float w1 = m31 ? *gptr(m31 + (size_t)r * J + c) : (g + c3 == c ? 1.f : 0.f);
                            a1[c3] = fmaf(w1, Q1[cc], a1[c3]);
                        }
                    }
                }
            }
#pragma unroll
            for (int c3 = 0; c3 < G3; ++c3) {
                if (g + c3 >= l3) break;
                out0[t * l3 + g + c3] = a0[c3];
                if constexpr (NB > 1) out1[t * l3 + g + c3] = a1[c3];
            }
        }
    }
}

// Split form of the finish (gram_split): thread (t, sl) = (tid % CHS, tid /
// CHS) sums, for pair q0 + t, the column tiles of channels [sl cps, (sl + 1)
// cps) (cps = ceil(J / GRAM_SPL)) and applies their columns of M (m3, or the
// identity); the GRAM_SPL slices' l3 values are then added through LDS (red:
// NB x GRAM_SPL x CHS x 16 floats) in slice order.
template <int NB>
__device__ __forceinline__ void finish_sketches_split(const Desc& d, int q0, int qn,
                                                      const float* __restrict__ P0, const float* __restrict__ m30,
                                                      float* out0, const float* __restrict__ P1,
                                                      const float* __restrict__ m31, float* out1, float* red) {
    constexpr int CHS = GRAM_CH_SPLIT, SPL = GRAM_SPL, G = 16, U = 8;
    const int tid = block_tid();
    const int L12 = d.l1 * d.l2, J = d.J, nt2 = d.n_i2t, l3 = d.l3;
    const int t = tid % CHS, sl = tid / CHS;
    const int cps = (J + SPL - 1) / SPL;
    const int c_lo = sl * cps, c_hi = min(J, c_lo + cps);
    float a0[G], a1[G];
#pragma unroll
    for (int c3 = 0; c3 < G; ++c3) { a0[c3] = 0.f; a1[c3] = 0.f; }
    if (t < qn) {
        const int q = q0 + t;
        for (int c = c_lo; c < c_hi; ++c) {
            float s0 = 0.f, s1 = 0.f;
            for (int t0 = 0; t0 < nt2; t0 += U) {
                float v0[U], v1[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const size_t off = ((size_t)c * nt2 + min(t0 + u, nt2 - 1)) * L12 + q;
                    v0[u] = *gptr(P0 + off);
                    if constexpr (NB > 1) v1[u] = *gptr(P1 + off);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool ok = t0 + u < nt2;
                    s0 += ok ? v0[u] : 0.f;
                    if constexpr (NB > 1) s1 += ok ? v1[u] : 0.f;
                }
            }
#pragma unroll
            for (int c3 = 0; c3 < G; ++c3) {
                if (c3 >= l3) break;
                const float w0 = m30 ? *gptr(m30 + (size_t)c3 * J + c) : (c3 == c ? 1.f : 0.f);
                a0[c3] = fmaf(w0, s0, a0[c3]);
                if constexpr (NB > 1) {
                    const float w1 = m31 ? *gptr(m31 + (size_t)c3 * J + c) : (c3 == c ? 1.f : 0.f);
                    a1[c3] = fmaf(w1, s1, a1[c3]);
                }
            }
        }
    }
#pragma unroll
    for (int c3 = 0; c3 < G; ++c3) {
        red[((size_t)sl * CHS + t) * G + c3] = a0[c3];
        if constexpr (NB > 1) red[((size_t)(SPL + sl) * CHS + t) * G + c3] = a1[c3];
    }
    __syncthreads();
    for (int e = tid; e < CHS * G; e += blockDim.x) {
        const int to = e / G, c3 = e % G;
        if (to >= qn || c3 >= l3) continue;
        float s0 = 0.f, s1 = 0.f;
        for (int s2 = 0; s2 < SPL; ++s2) {
            s0 += red[((size_t)s2 * CHS + to) * G + c3];
            if constexpr (NB > 1) s1 += red[((size_t)(SPL + s2) * CHS + to) * G + c3];
        }
        out0[to * l3 + c3] = s0;
        if constexpr (NB > 1) out1[to * l3 + c3] = s1;
    }
}

// Sum of 16 values over a wave in 17 shuffles: each of the first four levels
// halves the set a lane keeps (the lane bit of the level's offset picks the
// half), the last two add across neighbours, so that afterwards lanes
// 4k .. 4k + 3 hold the total of value k.
__device__ __forceinline__ void wave_sum16(float (&v)[16], int lane) {
#define RTG_HALVE(H, OFF)                                          \
    {                                                              \
        const bool up = (lane & (OFF)) != 0;                       \
        _Pragma("unroll") for (int k = 0; k < (H); ++k) {          \
            const float send = up ? v[k] : v[k + (H)];             \
            const float keep = up ? v[k + (H)] : v[k];             \
            v[k] = keep + __shfl_xor(send, (OFF), 64);             \
        }                                                          \
    }
    RTG_HALVE(8, 32) RTG_HALVE(4, 16) RTG_HALVE(2, 8) RTG_HALVE(1, 4)
#undef RTG_HALVE
    v[0] += __shfl_xor(v[0], 2, 64);
    v[0] += __shfl_xor(v[0], 1, 64);
}

// FROB_CHUNK elements of a tensor, FROB_PT consecutive ones per thread,
// from a buffer that reads zeros past its end.
constexpr int FROB_PT = FROB_CHUNK / 256;
static_assert(FROB_PT == 16, "two 8-element halves per thread");
__device__ __forceinline__ void frob_load(__amdgpu_buffer_rsrc_t r, bool bf, unsigned e, float (&x)[FROB_PT]) {
    if (bf) {
        typedef unsigned int u4v __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u4v w = __builtin_amdgcn_raw_buffer_load_b128(r, (e + 8u * h) * 2u, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                x[8 * h + 2 * q] = __uint_as_float(w[q] << 16);
                x[8 * h + 2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
            }
        }
    } else {
        typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const f4v w = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, (e + 4u * h) * 4u, 0, 0));
#pragma unroll
            for (int q = 0; q < 4; ++q) x[4 * h + q] = w[q];
        }
    }
}

// LDS of one sketched-Gram workgroup
struct GramSmem {
    double ds[2 * (MMAX + 2)];
    double wds[2 * (MMAX + 2)];   // this workgroup's shares
    double h1s[MMAX], hs[MMAX], gnew[MMAX], Gh1[MMAX], Gh[MMAX], cs_s[MMAX], sn_s[MMAX];
    double sG[GLDS * GLDS];       // stored block of G (symmetric), j <= GLDS
    double g_s;
    float s_s[4096];
    float s_v[4096];
    float red[4][16];
    int s_last;
};

// FROB: the sketch is the identity (unsketched global GMRES): the inner
// products are Frobenius products of the full tensors.  Each workgroup takes
// FROB_CHUNK elements of the problem's tensors and forms its shares of
// <V_i, W> and <V_i, V_j> (i <= j) and ||W||^2, reading every stored basis
// tensor once: the orthogonalisation traffic that a sketch avoids.
template <bool FROB>
__device__ __forceinline__ void gram_task(const Desc* __restrict__ descs, const int* __restrict__ starts,
                                          int count, int mode, int j, float* sketch_out, int b, GramSmem& sm) {
    float* s_s = sm.s_s;
    float* s_v = sm.s_v;
    double* ds = sm.ds;
    double* wds = sm.wds;
    double *h1s = sm.h1s, *hs = sm.hs, *gnew = sm.gnew, *Gh1 = sm.Gh1, *Gh = sm.Gh, *cs_s = sm.cs_s, *sn_s = sm.sn_s;
    double* sG = sm.sG;
    double& g_s = sm.g_s;
    int& s_last = sm.s_last;

    const int p = find_problem(starts, count, b);
    const Desc& d = descs[p];
    const int wgi = uniform_int(b - starts[p]);
    const int nwg = d.ntile[KIND_GRAM];
    if ((mode == GM_STEP || mode == GM_GK) && d.state[ST_ACTIVE] == 0) return;

    const int tid = block_tid(), lane = tid & 63, wave = tid >> 6;
    const int nitems = (mode == GM_STEP) ? j + 1 : 1;
    if constexpr (FROB) {
        // ---- Frobenius shares over elements [wgi FROB_CHUNK, (wgi + 1) FROB_CHUNK)
        float (*red)[16] = sm.red;
        const int es = d.bf16 ? 2 : 4;
        const int nb = (int)(d.n * 4);       // float32 tensors (W, R0); the host keeps n 4 < 2^31
        const unsigned e = (unsigned)wgi * FROB_CHUNK + (unsigned)tid * FROB_PT;
        const float* wsrc = (mode == GM_START) ? (const float*)d.R0src : d.W;
        const auto rw = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(wsrc), (short)0, nb, 0x00020000);
        float wv[FROB_PT];
        frob_load(rw, false, e, wv);
        float nw = 0.f;
#pragma unroll
        for (int u = 0; u < FROB_PT; ++u) nw = fmaf(wv[u], wv[u], nw);
        if (mode == GM_STEP) {
            auto basis = [&](int i) {
                return __builtin_amdgcn_make_buffer_rsrc((char*)d.V + (size_t)i * d.n * es, (short)0, (int)(d.n * es),
                                                         0x00020000);
            };
            float vj[FROB_PT];
            frob_load(basis(j - 1), d.bf16, e, vj);
            for (int i0 = 0; i0 < j; i0 += 8) {
                float acc[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) acc[k] = 0.f;
                float vb[2][FROB_PT];
                frob_load(basis(min(i0, j - 1)), d.bf16, e, vb[0]);
#pragma unroll
                for (int ii = 0; ii < 8; ++ii) {
                    if (ii + 1 < 8) frob_load(basis(min(i0 + ii + 1, j - 1)), d.bf16, e, vb[(ii + 1) & 1]);
                    __builtin_amdgcn_sched_barrier(0);   // one item ahead, no further
                    const bool live = i0 + ii < j;
#pragma unroll
                    for (int u = 0; u < FROB_PT; ++u) {
                        const float x = live ? vb[ii & 1][u] : 0.f;
                        acc[2 * ii] = fmaf(x, wv[u], acc[2 * ii]);
                        acc[2 * ii + 1] = fmaf(x, vj[u], acc[2 * ii + 1]);
                    }
                }
                wave_sum16(acc, lane);
                if ((lane & 3) == 0) red[wave][(lane >> 2) & 15] = acc[0];
                __syncthreads();
                if (tid < 16 && i0 + tid / 2 < j)
                    wds[2 * (i0 + tid / 2) + (tid & 1)] =
                        ((double)red[0][tid] + (double)red[1][tid]) + ((double)red[2][tid] + (double)red[3][tid]);
                __syncthreads();
            }
        }
        const double nws = wave_sum((double)nw);
        if (lane == 0) ds[wave] = nws;
        __syncthreads();
        if (tid == 0) {
            wds[2 * (nitems - 1)] = (ds[0] + ds[1]) + (ds[2] + ds[3]);
            wds[2 * (nitems - 1) + 1] = 0.0;
        }
    } else {
    const int L12 = d.l1 * d.l2, l3 = d.l3;
    const bool split = gram_split(l3, d.J, d.n_i2t);
    const int CH = (!split && d.gram_ch > 0) ? d.gram_ch : gram_pairs_per_block(l3, d.J, d.n_i2t);
    static_assert(2 * GRAM_SPL * GRAM_CH_SPLIT * 16 * sizeof(float) <= sizeof(double) * GLDS * GLDS,
                  "the split finish's reduction fits the G block's LDS");
    const int q0 = wgi * CH;
    const int qn = min(CH, L12 - q0);
    const int E = qn * l3;

    // in a step the W partials are those of S(Phi(V_j)) taken with the
    // composed first two matrices, so mode 3 is Om3 B^T
    // (Om3 B^T is banded when Om3 is the identity)
    const float* om3 = d.has_om3 ? d.om3 : nullptr;
    // (a general PSF: the W partials are those of W itself, mode 3 is Om3)
    // (the split form reduces through the LDS of the G block, which only the
    // tail fills, after the barrier below)
    // (the start step of an unnormalised V_1 reads that tensor's partials)
    const float* p_start = (mode == GM_START && d.lazy_v1) ? d.PV : d.PW;
    if (split) {
        if (mode == GM_STEP || mode == GM_GK)
            finish_sketches_split<2>(d, q0, qn, d.PW, d.st ? om3 : d.om3t, s_s, d.PV, om3, s_v, (float*)sG);
        else finish_sketches_split<1>(d, q0, qn, p_start, om3, s_s, nullptr, nullptr, nullptr, (float*)sG);
    } else if (mode == GM_STEP || mode == GM_GK)
        finish_sketches<2>(d, q0, qn, d.PW, d.st ? om3 : d.om3t, (d.st || d.has_om3) ? -1 : d.rB, s_s, d.PV, om3,
                           -1, s_v);
    else finish_sketches<1>(d, q0, qn, p_start, om3, -1, s_s, nullptr, nullptr, -1, nullptr);
    __syncthreads();
    if (mode == GM_STEP && j == 1 && d.lazy_v1) {
        // V_1 is stored unnormalised: S(V_1) and S(Phi(V_1)) scale by 1 / beta
        const float ib = (float)(1.0 / d.scal[SC_BETA]);
        for (int e = tid; e < E; e += 256) {
            s_s[e] *= ib;
            s_v[e] *= ib;
        }
        __syncthreads();
    }

    if (mode == GM_SKETCH_OUT) {
        const int l1 = d.l1, l2 = d.l2;
        for (int e = tid; e < E; e += 256) {
            const int q = q0 + e / l3, c3 = e % l3;
            const int a = q / l2, bb = q % l2;
            sketch_out[(size_t)a + (size_t)l1 * (bb + (size_t)l2 * c3)] = s_s[e];
        }
        return;
    }
    const size_t Lsz = (size_t)d.L;
    if (mode == GM_STEP || mode == GM_GK) {
        float* svj = d.SV + (size_t)(j - 1) * Lsz + (size_t)q0 * l3;
        for (int e = tid; e < E; e += 256) svj[e] = s_v[e];
    }
    if (mode == GM_GK) {
        // shares of ||s - cf S(Y)||^2 and ||s||^2; Y is the other side's
        // newest stored tensor (V_{c-1} for the U side, none at c = 1; U_c for
        // the V side) and cf its entry of the bidiagonal matrix (beta_c,
        // alpha_c), both written by earlier launches
        const int c = j, mm = d.m;
        const int prow = (d.gk == 1) ? c - 1 : c - 2;
        const double cf = prow < 0 ? 0.0
                                   : ((d.gk == 1) ? d.H[(size_t)(c - 1) * (mm + 1) + (c - 1)]
                                                  : d.H[(size_t)(c - 2) * (mm + 1) + (c - 1)]);
        const float* pv = d.SVx + (size_t)max(prow, 0) * Lsz + (size_t)q0 * l3;
        double a0 = 0.0, a1 = 0.0;
        for (int e = tid; e < E; e += 256) {
            const double se = s_s[e];
            const double t = se - (prow >= 0 ? cf * (double)pv[e] : 0.0);
            a0 += t * t;
            a1 += se * se;
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        if (lane == 0) {
            ds[2 * wave] = a0;
            ds[2 * wave + 1] = a1;
        }
        __syncthreads();
        if (tid == 0) {
            wds[0] = (ds[0] + ds[2]) + (ds[4] + ds[6]);
            wds[1] = (ds[1] + ds[3]) + (ds[5] + ds[7]);
        }
    }

    // ---- shares of the inner products (float64): <S(V_i), s> and
    // <S(V_i), S(V_j)> for the stored S(V_i), i < j - 1 (from global memory),
    // then the newest tensor S(V_j) and ||s||^2 from LDS.  Stored item i goes
    // to wave i % 4; a wave takes IG of its items per pass with EU elements
    // of each per lane, all loads in flight together (clamped indices,
    // masked: branch-free).
    const int nglob = (mode == GM_STEP) ? j - 1 : 0;
    if (mode != GM_GK) {
    constexpr int IG = 4, EU = 12;
    for (int it0 = wave; it0 < nglob; it0 += 4 * IG) {
        const float* svb = d.SV + (size_t)q0 * l3;
        double as[IG], av[IG];
#pragma unroll
        for (int u = 0; u < IG; ++u) { as[u] = 0.0; av[u] = 0.0; }
        for (int e0 = lane; e0 < E; e0 += 64 * EU) {
            float xv[IG][EU];
#pragma unroll
            for (int u = 0; u < IG; ++u)
#pragma unroll
                for (int eu = 0; eu < EU; ++eu)
                    xv[u][eu] = *gptr(svb + (size_t)min(it0 + 4 * u, nglob - 1) * Lsz + min(e0 + 64 * eu, E - 1));
#pragma unroll
            for (int eu = 0; eu < EU; ++eu) {
                const int e = e0 + 64 * eu;
                const bool ok = e < E;
                const double se = ok ? (double)s_s[min(e, E - 1)] : 0.0;
                const double ve = ok ? (double)s_v[min(e, E - 1)] : 0.0;
#pragma unroll
                for (int u = 0; u < IG; ++u) {
                    as[u] += (double)xv[u][eu] * se;
                    av[u] += (double)xv[u][eu] * ve;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < IG; ++u) {
            const double ra = wave_sum(as[u]);
            const double rv = wave_sum(av[u]);
            if (lane == 0 && it0 + 4 * u < nglob) {
                wds[(it0 + 4 * u) * 2 + 0] = ra;
                wds[(it0 + 4 * u) * 2 + 1] = rv;
            }
        }
    }
    if (wave == 3) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int e = lane; e < E; e += 64) {
            const double se = s_s[e], ve = s_v[e];
            a0 += se * se;
            a1 += ve * se;
            a2 += ve * ve;
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        if (lane == 0) {
            wds[(nitems - 1) * 2 + 0] = a0;
            wds[(nitems - 1) * 2 + 1] = 0.0;
            if (mode == GM_STEP) {
                wds[(j - 1) * 2 + 0] = a1;
                wds[(j - 1) * 2 + 1] = a2;
            }
        }
    }
    }   // GMRES shares

    }   // sketched shares

    // ---- the last workgroup of this problem finishes the step.  Wave 0
    // publishes the workgroup's shares with one release at agent scope (an
    // L2 write-back on this chip), then counts the workgroup in; the last one
    // to arrive acquires.  The stored S(V_j) is read only by later launches.
    __syncthreads();
    if (wave == 0) {
        double* dst = d.dots + (size_t)wgi * (MMAX + 2) * 2;
        for (int x = lane; x < 2 * nitems; x += 64) dst[x] = wds[x];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) {
            const int old = __hip_atomic_fetch_add(d.state + ST_COUNTER, 1, __ATOMIC_ACQUIRE,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            s_last = (old == nwg - 1);
        }
    }
    __syncthreads();
    if (!s_last) return;
    // Everything the rest reads from global memory is requested together:
    // the inner-product shares of all workgroups and, in a step with
    // j <= GLDS, the stored block G[0..j-2][0..j-2] (to LDS), the previous
    // plane rotations and g[j-1].
    const int m = d.m;
    const int ldg = m + 1;
    const int jm = j - 1;              // step: column index, also index of the newest basis tensor
    const bool g_lds = (mode == GM_STEP) && j <= GLDS && jm > 0;
    constexpr int GR = GLDS * GLDS / 256;
    double gblk[GR];
    if (g_lds) {
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            const int e = tid + 256 * r, i = e / GLDS, k = e % GLDS;
            gblk[r] = *gptr(d.G + (size_t)min(i, jm - 1) * ldg + min(k, jm - 1));
        }
    }
    double cs_r = 0.0, sn_r = 0.0, g_r = 0.0;
    if (mode == GM_STEP) {
        cs_r = *gptr(d.gv + min(tid, max(jm - 1, 0)));
        sn_r = *gptr(d.gv + m + min(tid, max(jm - 1, 0)));
        g_r = *gptr(d.gv + 2 * m + jm);
    }
    for (int x = tid; x < 2 * nitems; x += 256) {
        // fixed order over workgroups (deterministic); 16 loads in flight
        double part[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) part[u] = 0.0;
        const double* base = d.dots + (size_t)(x / 2) * 2 + (x & 1);
        for (int w0 = 0; w0 < nwg; w0 += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = load_coherent(base + (size_t)min(w0 + u, nwg - 1) * (MMAX + 2) * 2);
#pragma unroll
            for (int u = 0; u < 16; ++u) part[u] += (w0 + u < nwg) ? v[u] : 0.0;
        }
#pragma unroll
        for (int h = 8; h > 0; h >>= 1)
#pragma unroll
            for (int u = 0; u < h; ++u) part[u] += part[u + h];
        ds[x] = part[0];
    }
    if (g_lds) {
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            const int e = tid + 256 * r, i = e / GLDS, k = e % GLDS;
            if (i < jm && k < jm) sG[e] = gblk[r];
        }
    }
    if (mode == GM_STEP) {
        if (tid < jm) {                  // previous plane rotations, staged for the serial update
            cs_s[tid] = cs_r;
            sn_s[tid] = sn_r;
        }
        if (tid == 0) g_s = g_r;
    }
    __syncthreads();
    int* st = d.state;
    double* sc = d.scal;
    double* gvec = d.gv + 2 * m;       // rotated right-hand side g[0..m]
    if (mode == GM_START) {
        if (tid == 0) {
            st[ST_COUNTER] = 0;
            const double beta = sqrt(ds[0]);
            // a restart cycle (j > 0) starts only while ||R0||_Theta >= eps
            // (the residual test that ends the algorithm of Sec. 4.4)
            if (j > 0 && (st[ST_SKIP] != 0 || (d.stop_res > 0.0 && beta < d.stop_res))) {
                st[ST_SKIP] = 1;
                st[ST_ACTIVE] = 0;
                return;
            }
            sc[SC_BETA] = beta;
            gvec[0] = beta;
            if (!(beta > 0.0) || !isfinite(beta)) {
                st[ST_ACTIVE] = 0;
                st[ST_MEFF] = 0;
                st[ST_FLAGS] |= isfinite(beta) ? RTG_F_BREAKDOWN : RTG_F_NONFINITE;
                d.coef[MMAX + 1] = 0.f;
            } else {
                d.coef[MMAX + 1] = (float)(1.0 / beta);
            }
        }
        return;
    }
    if (mode == GM_GK) {
        if (tid == 0) {
            st[ST_COUNTER] = 0;
            const int c = j;
            const double nrm2 = ds[0];
            const double nrm = sqrt(nrm2 > 0.0 ? nrm2 : 0.0), rho = sqrt(ds[1]);
            const bool finite = isfinite(nrm) && isfinite(rho);
            double* Hc = d.H + (size_t)(c - 1) * (m + 1);
            if (d.gk == 2) {
                // alpha_c, the diagonal entry of column c; V_c = (Phi^T(U_c) - beta_c V_{c-1}) / alpha_c
                Hc[c - 1] = nrm;
                if (c >= 2) d.coef[c - 2] = (float)d.H[(size_t)(c - 2) * (m + 1) + (c - 1)];
                d.coef[MMAX + 1] = nrm > 0.0 ? (float)(1.0 / nrm) : 0.f;
                if (!finite) {
                    st[ST_FLAGS] |= RTG_F_NONFINITE;
                    st[ST_MEFF] = c - 1;
                    st[ST_ACTIVE] = 0;
                } else if (nrm <= d.bd_tol * rho) {
                    st[ST_FLAGS] |= RTG_F_BREAKDOWN;
                    st[ST_MEFF] = c - 1;
                    st[ST_ACTIVE] = 0;
                }
            } else {
                // beta_{c+1} completes column c = (alpha_c, beta_{c+1}) in rows c-1, c;
                // U_{c+1} = (Phi(V_c) - alpha_c U_c) / beta_{c+1}
                const double alpha = Hc[c - 1];
                Hc[c] = nrm;
                // Givens update: of the earlier rotations only the last one
                // meets a nonzero entry of this column
                double* cs = d.gv;
                double* sn = d.gv + m;
                double* Rc = d.R + (size_t)(c - 1) * m;
                for (int i = 0; i + 2 < c; ++i) Rc[i] = 0.0;
                double r_prev = alpha;
                if (c >= 2) {
                    Rc[c - 2] = sn[c - 2] * alpha;
                    r_prev = cs[c - 2] * alpha;
                }
                const double gj = gvec[c - 1];
                if (!finite) {
                    // the solve keeps the c - 1 complete columns: their
                    // rotations and g_1..g_c stay as the last step left them
                    st[ST_FLAGS] |= RTG_F_NONFINITE;
                    st[ST_MEFF] = c - 1;
                    st[ST_ACTIVE] = 0;
                    return;
                }
                const double rr = hypot(r_prev, nrm);
                const double cj = rr > 0.0 ? r_prev / rr : 1.0;
                const double sj = rr > 0.0 ? nrm / rr : 0.0;
                cs[c - 1] = cj;
                sn[c - 1] = sj;
                Rc[c - 1] = rr;
                gvec[c - 1] = cj * gj;
                gvec[c] = -sj * gj;
                const double res_ls = fabs(gvec[c]);
                sc[SC_RESLS] = res_ls;
                d.coef[c - 1] = (float)alpha;
                d.coef[MMAX + 1] = nrm > 0.0 ? (float)(1.0 / nrm) : 0.f;
                if (nrm <= d.bd_tol * rho) {
                    st[ST_FLAGS] |= RTG_F_BREAKDOWN;
                    st[ST_MEFF] = c;
                    st[ST_ACTIVE] = 0;
                } else if (d.stop_res > 0.0 && res_ls <= d.stop_res) {
                    st[ST_MEFF] = c;
                    st[ST_ACTIVE] = 0;
                } else if (c >= m && !d.keep_last) {
                    st[ST_MEFF] = c;
                    st[ST_ACTIVE] = 0;
                    if (d.stop_res > 0.0) st[ST_FLAGS] |= RTG_F_NOT_CONVERGED;
                } else {
                    st[ST_MEFF] = c;
                }
            }
        }
        return;
    }

    // ---- step j: classical Gram-Schmidt + reorthogonalisation in sketch space
    if (tid < j) {
        h1s[tid] = ds[2 * tid];
        gnew[tid] = ds[2 * tid + 1];
    }
    __syncthreads();
    if (tid < j) {
        d.G[(size_t)tid * ldg + jm] = gnew[tid];
        d.G[(size_t)jm * ldg + tid] = gnew[tid];
    }
    // Gh1 = G h1 and then Gh = G h with h = 2 h1 - G h1.  With the block of
    // G in LDS: a thread per row, k ascending (G is symmetric, so row i is
    // read as column i: neighbouring threads read neighbouring words).
    // Otherwise: each wave takes four rows at a time, lanes run along the row
    // (coalesced), wave reductions.
    auto gmatvec_lds = [&](const double* v, double* out, bool make_h) {
        for (int i = tid; i < j; i += 256) {
            double acc = 0.0;
            for (int k = 0; k < j; ++k) {
                double g = (k == jm) ? gnew[i] : sG[min(k, GLDS - 1) * GLDS + min(i, GLDS - 1)];
                g = (i == jm) ? gnew[k] : g;
                acc += g * v[k];
            }
            out[i] = acc;
            if (make_h) hs[i] = 2.0 * h1s[i] - acc;
        }
    };
    auto gmatvec = [&](const double* v, double* out, bool make_h) {
        if (g_lds || jm == 0) {
            gmatvec_lds(v, out, make_h);
            return;
        }
        for (int i0 = wave * 4; i0 < j; i0 += 16) {
            double acc4[4] = {0.0, 0.0, 0.0, 0.0};
            double gi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) gi[u] = gnew[min(i0 + u, j - 1)];
            for (int k = lane; k < j; k += 64) {
                const double vk = v[k];
                const double gk = gnew[k];
                double gl[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) gl[u] = *gptr(d.G + (size_t)min(i0 + u, j - 1) * ldg + k);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // row / column jm of G are the new entries (held in LDS)
                    const int i = min(i0 + u, j - 1);
                    double gik = (k == jm) ? gi[u] : gl[u];
                    gik = (i == jm) ? gk : gik;
                    acc4[u] += gik * vk;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u;
                const double r = wave_sum(acc4[u]);
                if (lane == 0 && i < j) {
                    out[i] = r;
                    if (make_h) hs[i] = 2.0 * h1s[i] - r;
                }
            }
        }
    };
    gmatvec(h1s, Gh1, true);
    __syncthreads();
    gmatvec(hs, Gh, false);
    __syncthreads();
    if (tid == 0) {
        st[ST_COUNTER] = 0;
        const double nrm2 = ds[2 * j];
        double hth1 = 0.0, hGh = 0.0;
        bool finite = isfinite(nrm2);
        for (int i = 0; i < j; ++i) {
            hth1 += hs[i] * h1s[i];
            hGh += hs[i] * Gh[i];
            finite = finite && isfinite(hs[i]);
        }
        const double hn2 = nrm2 - 2.0 * hth1 + hGh;
        const double hn = sqrt(hn2 > 0.0 ? hn2 : 0.0);
        const double rho = sqrt(nrm2);
        finite = finite && isfinite(hn);
        if (!finite) {
            // the solve keeps the jm complete columns: the rotations, R and
            // g_1..g_j stay as step jm left them (so gamma_j = g_j is the
            // residual of the jm-step problem)
            st[ST_FLAGS] |= RTG_F_NONFINITE;
            st[ST_MEFF] = jm;
            st[ST_ACTIVE] = 0;
            return;
        }
        // Hessenberg column
        double* Hc = d.H + (size_t)jm * (m + 1);
        for (int i = 0; i < j; ++i) Hc[i] = hs[i];
        Hc[j] = hn;
        // Givens update of the projected least-squares problem
        double* cs = d.gv;
        double* sn = d.gv + m;
        double* Rc = d.R + (size_t)jm * m;
        double r_prev = hs[0];
        for (int i = 0; i < jm; ++i) {
            const double a = r_prev, bnext = hs[i + 1];
            Rc[i] = cs_s[i] * a + sn_s[i] * bnext;
            r_prev = -sn_s[i] * a + cs_s[i] * bnext;
        }
        const double rr = hypot(r_prev, hn);
        const double cj = rr > 0.0 ? r_prev / rr : 1.0;
        const double sj = rr > 0.0 ? hn / rr : 0.0;
        cs[jm] = cj;
        sn[jm] = sj;
        Rc[jm] = rr;
        const double gj = g_s;
        gvec[jm] = cj * gj;
        gvec[j] = -sj * gj;
        const double res_ls = fabs(gvec[j]);
        sc[SC_RESLS] = res_ls;
        // coefficients of the orthogonalisation / normalisation (an
        // unnormalised stored V_1 = beta V_1 takes 1 / beta: in the scale at
        // step 1, where it is also the tensor the operator is applied to, and
        // in its own coefficient later)
        const double ib = d.lazy_v1 ? 1.0 / sc[SC_BETA] : 1.0;
        for (int i = 0; i < j; ++i) d.coef[i] = (float)(hs[i] * ((i == 0 && j >= 2) ? ib : 1.0));
        d.coef[MMAX + 1] = hn > 0.0 ? (float)((j == 1 ? ib : 1.0) / hn) : 0.f;
        // stopping decisions
        if (hn <= d.bd_tol * rho) {
            st[ST_FLAGS] |= RTG_F_BREAKDOWN;
            st[ST_MEFF] = j;
            st[ST_ACTIVE] = 0;
        } else if (d.stop_res > 0.0 && res_ls <= d.stop_res) {
            st[ST_MEFF] = j;
            st[ST_ACTIVE] = 0;
        } else if (j >= m && !d.keep_last) {
            st[ST_MEFF] = j;
            st[ST_ACTIVE] = 0;
            if (d.stop_res > 0.0) st[ST_FLAGS] |= RTG_F_NOT_CONVERGED;
        } else {
            st[ST_MEFF] = j;
        }
    }
}

}  // namespace rtg
