// One Arnoldi step over a column tile with the operator applied on the fly
// (Sec. 4.3; Phi of eq. (2)):
//
//   V_{j+1} = scale * (Phi(V_j) - sum_{i<=j} h_ij V_i),   scale = 1 / h_{j+1,j}
//
// plus the partial sketches of the stored V_{j+1} with (Om1, Om2) and with
// the composed (Om1 A1, Om2 A2), from which the next step's sketched inner
// products need S(V_{j+1}) and S(Phi(V_{j+1})).  W = Phi(V_j) is never
// stored: each workgroup recomputes it for its own tile from V_j.
//
// A workgroup owns output channel c and a strip of 32 columns (i2) over all
// I1 rows, walked in blocks of 64 rows.  Mode products commute, so per block
// it first mixes the input channels of c's band, U = sum_k B[k, c] V_j[k]
// (on a slab with an R-wide halo, zeros outside the tensor), then blurs U
// along i1 and along i2 with the band rows staged in LDS (wave-uniform
// coefficients), which gives the W tile in registers.  The tile goes through
// LDS to a layout where each lane owns eight consecutive rows of one column
// for the multi-AXPY (16-byte loads of the basis, software-pipelined over
// the terms, the first two terms in flight during the blur), the result is
// scaled, rounded (bfloat16 basis) and stored, and it is contracted on MFMA
// against the stacked [Om1 ; Om1 A1] rows of the block (as in the tile
// kernel).  After the last block the mode-2 contraction writes the partials.
#include "rtg_internal.h"

namespace rtg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int STEP_T1 = 64;          // rows per block
constexpr unsigned STEP_OOB = 0x20000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t step_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

template <int R, bool BB, int RPW>
struct StepSmem {
    static constexpr int T1 = STEP_T1, TC = TILE_TC;
    static constexpr int SR = T1 + 2 * R, SRP = SR + 1, SC = TC + 2 * R, ZRP = T1 + 1;
    static constexpr int WP = ((2 * R + 1) + 3) / 4 * 4;
    static constexpr int WTP = T1 + 4;                  // W tile, column-major
    static constexpr int XP = BB ? T1 + 8 : T1 + 4;     // MFMA B tile, column-major
    static constexpr int YP = TC + 1;
    static constexpr int U1 = SC * SRP + SC * ZRP;      // slab + Z (floats)
    static constexpr int UY = 64 * RPW * YP;            // mode-1 results (floats)
    static constexpr int UN = U1 > UY ? U1 : UY;
    static constexpr int XB = BB ? TC * XP * 2 : TC * XP * 4;
};

template <int R, bool BB, int RPW>
__global__ void __launch_bounds__(256) k_step(const Desc* __restrict__ descs, const int* __restrict__ starts,
                                              int count, int j) {
    using SM = StepSmem<R, BB, RPW>;
    constexpr int T1 = SM::T1, TC = SM::TC;
    constexpr int SR = SM::SR, SRP = SM::SRP, SC = SM::SC, ZRP = SM::ZRP, WP = SM::WP;
    constexpr int WTP = SM::WTP, XP = SM::XP, YP = SM::YP;
    constexpr int SRH = SR / 2;                         // row pairs of the slab
    constexpr int NLP = (SRH * SC + 255) / 256;         // slab row pairs per lane
    constexpr int KG = 3;                               // input channels loaded together
    constexpr int KBR = BB ? 32 : 16;                   // rows per MFMA K-block
    constexpr int NST = BB ? 1 : 2;                     // 16-byte loads per lane per term

    __shared__ float coef_s[MMAX + 2];
    __shared__ __attribute__((aligned(16))) float su[SM::UN];
    __shared__ float A1c[T1 * WP];
    __shared__ float A2c[TC * WP];
    __shared__ __attribute__((aligned(16))) unsigned char sx[SM::XB];
    float* S = su;                      // [SC][SRP] mixed slab
    float* Z = su + SC * SRP;           // [SC][ZRP] after the i1 pass
    float* Wt = su;                     // [TC][WTP] W tile (reuses the slab)
    float* Ys = su;                     // [16 NRT][YP] (after the last block)
    bf16_t* Xh = (bf16_t*)sx;
    float* Xf = (float*)sx;

    const int b = blockIdx.x;
    const int p = find_problem(starts, count, b);
    const Desc& d = descs[p];
    const int tile = b - starts[p];
    if (d.state[ST_ACTIVE] == 0) return;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15, kq = lane >> 4;
    const int I1 = d.I1, I2 = d.I2, J = d.J;
    const int l1 = d.l1, l2 = d.l2;
    const int t2 = tile % d.n_i2t, c = tile / d.n_i2t;
    const int i20 = t2 * TC;
    const int ncol = min(TC, I2 - i20);
    const int r1 = d.r1, r2 = d.r2, rB = d.rB;
    const int w1 = 2 * r1 + 1, w2 = 2 * r2 + 1, wB = 2 * rB + 1;
    const int klo = max(0, c - rB), khi = min(J, c + rB + 1);
    const size_t plane = (size_t)I1 * I2;
    const size_t es = BB ? 2 : 4;
    const size_t tile_off = (size_t)c * plane + (size_t)i20 * I1;
    const int tile_elems = ncol * I1;
    const char* vj = (const char*)d.V + (size_t)(j - 1) * d.n * es;   // V_j, source of Phi

    const int nterms = j;
    for (int i = tid; i < nterms; i += 256) coef_s[i] = d.coef[i];
    const float scale = d.coef[MMAX + 1];
    for (int e = tid; e < TC * WP; e += 256) {
        const int col = e / WP, t = e % WP, dd = t - R;
        const int i2 = i20 + col;
        A2c[e] = (t <= 2 * R && dd >= -r2 && dd <= r2 && i2 < I2) ? *gptr(d.a2 + (size_t)i2 * w2 + r2 + dd) : 0.f;
    }

    const int RT = (l1 + 15) >> 4;
    const int NRT = 2 * RT;
    f4 acc[RPW][2];
#pragma unroll
    for (int u = 0; u < RPW; ++u)
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[u][g] = f4{0.f, 0.f, 0.f, 0.f};

    // slab element e = tid + 256 it: row e % SR, column e / SR (rows fastest:
    // coalesced), 32-bit offsets within a channel plane, in-tensor bits
    const int ac = tid >> 3, ar = 8 * (tid & 7);     // AXPY lane: column ac, rows ar .. ar + 7

    const int nrb = (I1 + T1 - 1) / T1;
    unsigned soff[NLP];
    // (buffer loads: a uniform channel base and 32-bit per-lane offsets,
    // always inside the channel plane)
    auto load_slab = [&](int k, unsigned (*dst)[BB ? 1 : 2]) {
        const auto rs = step_rsrc(vj + (size_t)k * plane * es, (int)(plane * es));
#pragma unroll
        for (int it = 0; it < NLP; ++it) {
            if constexpr (BB) {
                dst[it][0] = __builtin_amdgcn_raw_buffer_load_b32(rs, soff[it], 0, 0);
            } else {
                const auto w2v = __builtin_amdgcn_raw_buffer_load_b64(rs, soff[it], 0, 0);
                dst[it][0] = w2v[0];
                dst[it][1] = w2v[1];
            }
        }
    };
    auto mix = [&](float (*u)[2], const unsigned (*src)[BB ? 1 : 2], float w) {
#pragma unroll
        for (int it = 0; it < NLP; ++it) {
            if constexpr (BB) {
                u[it][0] = fmaf(w, __uint_as_float(src[it][0] << 16), u[it][0]);
                u[it][1] = fmaf(w, __uint_as_float(src[it][0] & 0xffff0000u), u[it][1]);
            } else {
                u[it][0] = fmaf(w, __uint_as_float(src[it][0]), u[it][0]);
                u[it][1] = fmaf(w, __uint_as_float(src[it][1]), u[it][1]);
            }
        }
    };
    auto bweight = [&](int k) {
        const int kc = min(k, khi - 1);
        const float bkc = *gptr(d.bb + (size_t)kc * wB + rB + (c - kc));
        return k < khi ? bkc : 0.f;
    };

    for (int rb = 0; rb < nrb; ++rb) {
        const int i10 = rb * T1;
        __syncthreads();                  // previous block: LDS reads done (A1c, S, Z, Wt, X)
        // ---- slab offsets: a lane loads two consecutive rows (the slab starts
        // on an even row and I1 is even, so a pair is inside the tensor or outside)
        unsigned sok = 0;
#pragma unroll
        for (int it = 0; it < NLP; ++it) {
            const int e = tid + 256 * it;
            const int rp = e % SRH, col = e / SRH;
            const int i1 = i10 - R + 2 * rp, i2 = i20 - R + col;
            sok |= (unsigned)((e < SRH * SC) & (i1 >= 0) & (i1 < I1) & (i2 >= 0) & (i2 < I2)) << it;
            soff[it] = (unsigned)(min(max(i2, 0), I2 - 1) * I1 + min(max(i1, 0), I1 - 2)) * (unsigned)es;
        }
        // the first two multi-AXPY terms of this block go in flight now
        const unsigned aoff = (ac < ncol && i10 + ar < I1) ? (unsigned)(ac * I1 + i10 + ar) * (unsigned)es : STEP_OOB;
        auto load_term = [&](int i, u4* v) {
            const auto rv = step_rsrc((const char*)d.V + ((size_t)i * d.n + tile_off) * es, tile_elems * (int)es);
#pragma unroll
            for (int s2 = 0; s2 < NST; ++s2) v[s2] = __builtin_amdgcn_raw_buffer_load_b128(rv, aoff + 16u * s2, 0, 0);
        };
        u4 va[NST], vb[NST];
        if (nterms > 0) load_term(0, va);
        if (nterms > 1) load_term(1, vb);
        // ---- band rows of the block, and the mixed slab
        //      U = sum_k B[k, c] V_j[k] (zero outside the tensor)
        for (int e = tid; e < T1 * WP; e += 256) {
            const int row = e / WP, t = e % WP, dd = t - R;
            const int i1 = i10 + row;
            A1c[e] = (t <= 2 * R && dd >= -r1 && dd <= r1 && i1 < I1) ? *gptr(d.a1 + (size_t)i1 * w1 + r1 + dd) : 0.f;
        }
        float u[NLP][2];
#pragma unroll
        for (int it = 0; it < NLP; ++it) { u[it][0] = 0.f; u[it][1] = 0.f; }
        for (int k0 = klo; k0 < khi; k0 += KG) {
            unsigned v[KG][NLP][BB ? 1 : 2];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) load_slab(min(k0 + kk, khi - 1), v[kk]);
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) mix(u, v[kk], bweight(k0 + kk));
        }
#pragma unroll
        for (int it = 0; it < NLP; ++it) {
            const int e = tid + 256 * it;
            if (e < SRH * SC) {
                const bool ok = (sok >> it) & 1u;
                float* sp = S + (e / SRH) * SRP + 2 * (e % SRH);
                sp[0] = ok ? u[it][0] : 0.f;
                sp[1] = ok ? u[it][1] : 0.f;
            }
        }
        const int nkb = (min(T1, I1 - i10) + KBR - 1) / KBR;
        struct AF {
            u4 h, l;
        };
        auto load_a = [&](int kb, AF* A) {
            const int row = i10 + kb * KBR + (BB ? 8 : 4) * kq;
            const int rowc = min(row, I1 - (BB ? 8 : 4));
#pragma unroll
            for (int u2 = 0; u2 < RPW; ++u2) {
                const int t = wave + 4 * u2;
                const int half = (t >= RT && t < NRT) ? 1 : 0;
                const int a = 16 * (t - half * RT) + m16;
                const unsigned msk = 0u - (unsigned)((a < l1) & (row < I1) & (t < NRT));
                const unsigned off = (unsigned)(min(a, l1 - 1) * I1 + rowc);
                if constexpr (BB) {
                    const char* base = (const char*)(half ? d.om1th : d.om1h);
                    const char* lob = base + (half ? (size_t)l1 * I1 * 2 : 0);
                    A[u2].h = *gptr((const u4*)(base + off * 2u)) & msk;
                    A[u2].l = *gptr((const u4*)(lob + off * 2u)) & (half ? msk : 0u);
                } else {
                    const char* base = (const char*)(half ? d.om1t : d.om1);
                    A[u2].h = *gptr((const u4*)(base + off * 4u)) & msk;
                }
            }
        };
        __syncthreads();
        // ---- i1 pass: Z[col][row] = sum_d A1[i1, i1 + d] U[col][row + R + d]
        if (lane < SC) {
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                const int rbase = wave * 16 + blk * 8;
                float in[8 + 2 * R];
#pragma unroll
                for (int e = 0; e < 8 + 2 * R; ++e) in[e] = S[lane * SRP + rbase + e];
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const float* cr = A1c + (rbase + o) * WP;
                    float s2 = 0.f;
#pragma unroll
                    for (int t = 0; t <= 2 * R; ++t) s2 = fmaf(cr[t], in[o + t], s2);
                    Z[lane * ZRP + rbase + o] = s2;
                }
            }
        }
        __syncthreads();
        // ---- i2 pass (lane = row, wave = eight columns), W tile to LDS
        {
            float in2[8 + 2 * R];
#pragma unroll
            for (int e = 0; e < 8 + 2 * R; ++e) in2[e] = Z[(wave * 8 + e) * ZRP + lane];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const float* cr = A2c + (wave * 8 + o) * WP;
                float s2 = 0.f;
#pragma unroll
                for (int t = 0; t <= 2 * R; ++t) s2 = fmaf(cr[t], in2[o + t], s2);
                Wt[(wave * 8 + o) * WTP + lane] = s2;
            }
        }
        __syncthreads();
        // ---- multi-AXPY on eight rows of one column per lane
        float x[8];
        {
            const f4 w0 = *(const f4*)(Wt + ac * WTP + ar);
            const f4 w1v = *(const f4*)(Wt + ac * WTP + ar + 4);
            x[0] = w0[0]; x[1] = w0[1]; x[2] = w0[2]; x[3] = w0[3];
            x[4] = w1v[0]; x[5] = w1v[1]; x[6] = w1v[2]; x[7] = w1v[3];
        }
        auto apply_term = [&](float ci, const u4* v) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (BB) {
                    x[2 * q] = fmaf(-ci, __uint_as_float(v[0][q] << 16), x[2 * q]);
                    x[2 * q + 1] = fmaf(-ci, __uint_as_float(v[0][q] & 0xffff0000u), x[2 * q + 1]);
                } else {
                    x[q] = fmaf(-ci, __uint_as_float(v[0][q]), x[q]);
                    x[4 + q] = fmaf(-ci, __uint_as_float(v[1][q]), x[4 + q]);
                }
            }
        };
        for (int i = 0; i < nterms; i += 2) {
            apply_term(coef_s[i], va);
            if (i + 2 < nterms) load_term(i + 2, va);
            if (i + 1 < nterms) {
                apply_term(coef_s[i + 1], vb);
                if (i + 3 < nterms) load_term(i + 3, vb);
            }
        }
        const bool aok = aoff != STEP_OOB;
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = aok ? x[q] * scale : 0.f;
        const auto rd = step_rsrc((const char*)d.V + ((size_t)j * d.n + tile_off) * es, tile_elems * (int)es);
        if constexpr (BB) {
            u4 pk;
#pragma unroll
            for (int q = 0; q < 4; ++q) pk[q] = (unsigned)f2bf(x[2 * q]) | ((unsigned)f2bf(x[2 * q + 1]) << 16);
            __builtin_amdgcn_raw_buffer_store_b128(pk, rd, aoff, 0, 0);
            *(u4*)(Xh + ac * XP + ar) = pk;
        } else {
            const u4 p0 = u4{__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]), __float_as_uint(x[3])};
            const u4 p1 = u4{__float_as_uint(x[4]), __float_as_uint(x[5]), __float_as_uint(x[6]), __float_as_uint(x[7])};
            __builtin_amdgcn_raw_buffer_store_b128(p0, rd, aoff, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(p1, rd, aoff + 16u, 0, 0);
            *(f4*)(Xf + ac * XP + ar) = f4{x[0], x[1], x[2], x[3]};
            *(f4*)(Xf + ac * XP + ar + 4) = f4{x[4], x[5], x[6], x[7]};
        }
        __syncthreads();
        // ---- mode-1 contraction of this block on MFMA (stacked rows [Om1 ; Om1 A1])
        auto mfma_block = [&](int kb, const AF* A) {
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int col = 16 * g + m16;
                if constexpr (BB) {
                    const u4 bh = *(const u4*)(Xh + col * XP + kb * KBR + 8 * kq);
#pragma unroll
                    for (int u2 = 0; u2 < RPW; ++u2) {
                        const int t = wave + 4 * u2;
                        if (t >= NRT) break;
                        acc[u2][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf8, A[u2].h), __builtin_bit_cast(bf8, bh), acc[u2][g], 0, 0, 0);
                        if (t >= RT)
                            acc[u2][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf8, A[u2].l), __builtin_bit_cast(bf8, bh), acc[u2][g], 0, 0, 0);
                    }
                } else {
                    const f4 bv = *(const f4*)(Xf + col * XP + kb * KBR + 4 * kq);
#pragma unroll
                    for (int u2 = 0; u2 < RPW; ++u2) {
                        const int t = wave + 4 * u2;
                        if (t >= NRT) break;
                        const f4 av = __builtin_bit_cast(f4, A[u2].h);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[u2][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], acc[u2][g], 0, 0, 0);
                    }
                }
            }
        };
        AF A0[RPW], A1[RPW];
        load_a(0, A0);
        for (int kb = 0; kb < nkb; kb += 2) {
            if (kb + 1 < nkb) load_a(kb + 1, A1);
            mfma_block(kb, A0);
            if (kb + 1 < nkb) {
                if (kb + 2 < nkb) load_a(kb + 2, A0);
                mfma_block(kb + 1, A1);
            }
        }
    }

    // ---- mode-1 results to LDS, then the mode-2 contraction
    __syncthreads();
#pragma unroll
    for (int u2 = 0; u2 < RPW; ++u2) {
        const int t = wave + 4 * u2;
        if (t >= NRT) break;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) Ys[(16 * t + 4 * kq + i) * YP + 16 * g + m16] = acc[u2][g][i];
    }
    __syncthreads();
    const int RT2 = (l2 + 15) >> 4;
    for (int tt = wave; tt < NRT * RT2; tt += 4) {
        const int t = tt / RT2, rt2 = tt % RT2;
        const int half = t >= RT ? 1 : 0;
        const float* om2x = half ? d.om2t : d.om2;
        float* P = (half ? d.PW : d.PV) + (size_t)tile * l1 * l2;
        const int bcol = 16 * rt2 + m16;
        float Bv[TC / 4];
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks) {
            const int k = 4 * ks + kq;
            const float v = *gptr(om2x + (size_t)min(bcol, l2 - 1) * I2 + i20 + min(k, ncol - 1));
            Bv[ks] = (bcol < l2 && k < ncol) ? v : 0.f;
        }
        f4 pacc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks)
            pacc = __builtin_amdgcn_mfma_f32_16x16x4f32(Ys[(16 * t + m16) * YP + 4 * ks + kq], Bv[ks], pacc, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ar2 = 16 * (t - half * RT) + 4 * kq + i;
            if (ar2 < l1 && bcol < l2) *gptr_w(P + (size_t)ar2 * l2 + bcol) = pacc[i];
        }
    }
}

// Only the bfloat16-basis variants are built: with a float32 basis the
// solver forms W with the operator kernel and uses the tile kernel (faster
// there, see the launch sequence).
hipError_t launch_step(const Desc* d, const int* starts, int count, int total_tiles, int j, int rmax,
                       int basis_bf16, int l1max, hipStream_t s) {
    if (!basis_bf16) return hipErrorInvalidValue;
    const int tier = rmax <= 4 ? 4 : (rmax <= 8 ? 8 : 12);
    const bool small = 2 * ((l1max + 15) / 16) <= 8;
#define RTG_STEP(RR, RPV) \
    hipLaunchKernelGGL((k_step<RR, true, RPV>), dim3(total_tiles), dim3(256), 0, s, d, starts, count, j)
#define RTG_STEP_R(RR) if (small) RTG_STEP(RR, 2); else RTG_STEP(RR, 4);
    if (tier == 4) { RTG_STEP_R(4) } else if (tier == 8) { RTG_STEP_R(8) } else { RTG_STEP_R(12) }
#undef RTG_STEP_R
#undef RTG_STEP
    return hipGetLastError();
}

}  // namespace rtg
